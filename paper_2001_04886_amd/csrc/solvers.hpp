// solvers.hpp -- internal entry points of the solver drivers.
#pragma once

#include <cstddef>

#include "../../include/sstep.h"
#include "launch.hpp"

namespace sstep {

size_t gmres_workspace_bytes(const sstep_stencil& A, int s, int m, int precision);
int gmres_solve_impl(Ctx& c, const sstep_stencil& A, const double* f, double* x, int s, int m,
                     double tol, const sstep_options& opt, sstep_info* info, void* ws,
                     size_t ws_bytes);

size_t omin_workspace_bytes(const sstep_stencil& A, int s, int k);
int omin_solve_impl(Ctx& c, const sstep_stencil& A, const double* f, double* x, int s, int k,
                    double tol, const sstep_options& opt, sstep_info* info, void* ws,
                    size_t ws_bytes);

size_t batched_workspace_bytes(int nsys, const sstep_stencil* A, int s, int m, int nslots);
int batched_slots(int nsys, int wgs_per_cu, int team);
int batched_plan_create(void** out, int nsys, const sstep_stencil* A, const double* const* f,
                        double* const* x, int s, int m, double tol, const sstep_options& opt);
int batched_plan_execute(void* plan, sstep_info* info, double* ms_out);
void batched_plan_destroy(void* plan);

}  // namespace sstep
