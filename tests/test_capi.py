"""C-ABI boundary checks that need no GPU: the library loads, exports every
symbol the header declares, and rejects invalid arguments before launching."""
import ctypes as C
import os
import re

import pytest

from paper_2001_04886_amd import sstep as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "sstep.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sstep_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_binding_exports():
    assert header_functions() == sorted(S.EXPORTS)


def test_library_loads_and_exports_every_symbol():
    lib = S.load()
    for name in header_functions():
        assert hasattr(lib, name), name


def test_status_strings():
    for st in (0, 1, -1, -2, -3, -4, -5):
        assert len(S.status_string(st)) > 3
    assert S.status_string(99) == "unknown status"


def test_workspace_sizing_and_argument_checks():
    A = S.Stencil(3, 256, 256, 256, (1.0,) * 7)
    nb = S.workspace_bytes(A, S.METHOD_GMRES, 8, 40)
    N = 256 ** 3
    assert nb >= 321 * N * 8            # the basis: m*s+1 FP64 columns
    assert nb < 321 * N * 8 * 1.01
    nb32 = S.workspace_bytes(A, S.METHOD_GMRES, 8, 40, S.MIXED)
    assert 321 * N * 4 <= nb32 < nb
    assert S.workspace_bytes(A, S.METHOD_OMIN, 8, 8) >= (2 * 64 + 9) * N * 8
    assert S.workspace_bytes(A, S.METHOD_GMRES, 0, 40) == 0
    assert S.workspace_bytes(A, S.METHOD_GMRES, 17, 40) == 0
    assert S.workspace_bytes(A, S.METHOD_GMRES, 8, 300) == 0   # m*s > 2048
    assert S.workspace_bytes(A, S.METHOD_OMIN, 8, 65) == 0
    assert S.workspace_bytes(A, S.METHOD_OMIN, 8, 8, S.MIXED) == 0
    bad = S.Stencil(4, 8, 8, 8, (1.0,) * 7)
    assert S.workspace_bytes(bad, S.METHOD_GMRES, 4, 4) == 0


def test_size_limits_without_launching():
    # grids up to 2^31 - 1 points are accepted (1290^3), larger ones rejected
    # (1291^3); empty grids and empty kernel operands are rejected
    big = S.Stencil(3, 1290, 1290, 1290, (6.0, -1, -1, -1, -1, -1, -1))
    assert S.workspace_bytes(big, S.METHOD_GMRES, 2, 2) > 5 * 1290 ** 3 * 8
    over = S.Stencil(3, 1291, 1291, 1291, (6.0, -1, -1, -1, -1, -1, -1))
    assert S.workspace_bytes(over, S.METHOD_GMRES, 2, 2) == 0
    assert S.workspace_bytes(S.Stencil(2, 46341, 46341, 1, (4.0, -1, -1, -1, -1, 0, 0)),
                             S.METHOD_GMRES, 2, 2) == 0
    lib = S.load()
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    oc = over.c_struct()
    assert lib.sstep_gmres_solve(C.byref(oc), fake, fake, 2, 2, 1e-8, None, None) == -1
    assert lib.sstep_omin_solve(C.byref(oc), fake, fake, 2, 2, 1e-8, None, None) == -1
    assert lib.sstep_stencil_apply(C.byref(oc), fake, C.c_void_p(0x2000), None) == -1
    for nx, ny, nz in [(0, 5, 5), (5, 0, 5), (5, 5, 0)]:
        e = S.Stencil(3, nx, ny, nz, (6.0, -1, -1, -1, -1, -1, -1))
        assert S.workspace_bytes(e, S.METHOD_GMRES, 2, 2) == 0
    assert lib.sstep_kernel_gram(fake, 0, 3, fake, 0, 3, 0, fake, None) == -1          # N = 0
    assert lib.sstep_kernel_gram(fake, 64, 0, fake, 64, 3, 64, fake, None) == -1       # no columns
    assert lib.sstep_kernel_gram(fake, 1 << 31, 3, fake, 1 << 31, 3, 1 << 31, fake, None) == -1
    assert lib.sstep_kernel_update(fake, 0, 2, fake, 0, 2, fake, 0, None) == -1        # N = 0
    assert lib.sstep_kernel_update(fake, 64, 2, fake, 64, 0, fake, 64, None) == -1     # no outputs


def test_solvers_reject_bad_arguments_without_launching():
    lib = S.load()
    A = S.Stencil(2, 8, 8, 1, (4.0, -1, -1, -1, -1, 0, 0)).c_struct()
    info = S.InfoC()
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.sstep_gmres_solve(C.byref(A), fake, fake, 0, 4, 1e-8, None, C.byref(info)) == -1
    assert info.status == -1
    assert lib.sstep_gmres_solve(C.byref(A), fake, fake, 4, 4, -1.0, None, None) == -1
    assert lib.sstep_gmres_solve(C.byref(A), None, fake, 4, 4, 1e-8, None, None) == -1
    assert lib.sstep_omin_solve(C.byref(A), fake, fake, 4, 0, 1e-8, None, None) == -1
    o = S.OptionsC()
    lib.sstep_default_options(C.byref(o))
    o.precision = 1
    assert lib.sstep_omin_solve(C.byref(A), fake, fake, 4, 4, 1e-8, C.byref(o), None) == -1
    o.precision = 0
    o.basis = 7
    assert lib.sstep_gmres_solve(C.byref(A), fake, fake, 4, 4, 1e-8, C.byref(o), None) == -1
    Bad = S.Stencil(2, 0, 8, 1, (4.0, -1, -1, -1, -1, 0, 0)).c_struct()
    assert lib.sstep_gmres_solve(C.byref(Bad), fake, fake, 4, 4, 1e-8, None, None) == -1
    assert lib.sstep_stencil_apply(C.byref(A), fake, fake, None) == -1   # x == y
    assert lib.sstep_kernel_gram(fake, 10, 3, fake, 10, 17, 10, fake, None) == -1


def test_network_entry_points_validate_without_launching():
    lib = S.load()
    assert lib.sstep_cnn_param_count() == 19393
    # workspace: training needs the gradient buffers, inference the fallback test
    assert lib.sstep_cnn_workspace_bytes(0, 8, 8, 1) == 0
    tr = lib.sstep_cnn_workspace_bytes(4, 64, 48, 1)
    inf = lib.sstep_cnn_workspace_bytes(4, 64, 48, 0)
    assert tr > inf > 4 * 64 * 48 * (4 + 3 * 64)
    o = S.OptionsC()
    lib.sstep_default_options(C.byref(o))
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.sstep_cnn_forward(fake, 1.0, 0, 8, 8, fake, fake, None, fake, C.byref(o)) == S.ERR_ARG
    assert lib.sstep_cnn_forward(fake, 0.0, 1, 8, 8, fake, fake, None, fake, C.byref(o)) == S.ERR_ARG
    assert lib.sstep_cnn_forward(fake, 1.0, 1, 8, 8, fake, fake, None, None, C.byref(o)) == S.ERR_ARG
    assert lib.sstep_cnn_adam(fake, fake, fake, fake, 0, 1e-3, C.byref(o)) == S.ERR_ARG
    assert lib.sstep_cnn_train_step(fake, fake, fake, 1, -1.0, 1.0, 1, 8, 8, fake, fake, fake,
                                    None, C.byref(o)) == S.ERR_ARG
    A = S.Stencil(3, 8, 8, 8, (6.0, -1, -1, -1, -1, -1, -1)).c_struct()  # x0 guess is 2-D only
    used = C.c_int(7)
    assert lib.sstep_x0_predict(fake, 1.0, C.byref(A), fake, fake, fake, 1, C.byref(used),
                                C.byref(o)) == S.ERR_ARG
    assert used.value == 0


def test_batch_options_validated_without_launching():
    lib = S.load()
    A = (S.StencilC * 2)(*[S.Stencil(2, 10, 10, 1, (4.0, -1, -1, -1, -1, 0, 0)).c_struct()] * 2)
    f = (C.c_void_p * 2)(0x1000, 0x2000)
    x = (C.c_void_p * 2)(0x3000, 0x4000)
    plan = C.c_void_p()
    # Gram column tile: 2 or 4 for s <= 4, 1 or 2 for s <= 8
    for field, bad, s in (("batch_team", 3, 4), ("batch_threads", 300, 4), ("batch_wgs_per_cu", 5, 4),
                          ("batch_gram_cols", 1, 4), ("batch_gram_cols", 3, 4),
                          ("batch_gram_cols", 4, 8)):
        o = S.OptionsC()
        lib.sstep_default_options(C.byref(o))
        setattr(o, field, bad)
        assert lib.sstep_batch_plan_create(C.byref(plan), 2, A, f, x, s, 8, 1e-8, C.byref(o)) == S.ERR_ARG
    o = S.OptionsC()
    lib.sstep_default_options(C.byref(o))
    assert lib.sstep_batch_plan_create(C.byref(plan), 2, A, f, x, 9, 8, 1e-8, C.byref(o)) == S.ERR_ARG
    misaligned = (C.c_void_p * 2)(0x1008, 0x2000)
    assert lib.sstep_batch_plan_create(C.byref(plan), 2, A, misaligned, x, 4, 8, 1e-8,
                                       C.byref(o)) == S.ERR_ARG


def test_tuner_table_lookup(tmp_path, monkeypatch):
    import json
    from paper_2001_04886_amd import tune as TU
    monkeypatch.setattr(TU, "_arch", lambda: "gfx950")
    st = [S.Stencil(2, 32, 32), S.Stencil(2, 40, 40)]
    path = str(tmp_path / "t.json")
    assert TU.lookup(st, 4, 30, path) is None
    key = TU.batch_key(st, 4, 30)
    assert key == "gfx950|n2|N2624|max1600|s4|m30"
    # a record without the Gram column tile gives tile 0 (the library default)
    json.dump({key: {"threads": 512, "wgs_per_cu": 1, "team": 2}}, open(path, "w"))
    assert TU.lookup(st, 4, 30, path) == (512, 1, 2, 0)
    json.dump({key: {"threads": 512, "wgs_per_cu": 1, "team": 2, "gram_cols": 2}}, open(path, "w"))
    assert TU.lookup(st, 4, 30, path) == (512, 1, 2, 2)
    assert TU.lookup(st, 8, 30, path) is None
    assert TU.gram_cols(4, TU.NARROW) == 2 and TU.gram_cols(8, TU.NARROW) == 1
    assert TU.gram_cols(4, 0) == 0
    # a record without the team size (older table layout) is not used
    json.dump({key: {"threads": 512, "wgs_per_cu": 1}}, open(path, "w"))
    assert TU.lookup(st, 4, 30, path) is None


def test_learned_model_parameters_layout():
    from paper_2001_04886_amd import learn as LN
    p = LN.init_params(3)
    assert p.dtype.name == "float32" and p.size == 19393
    # biases start at zero: b1 (32 after 576 weights), b2, b3 (32 each), b4 (1)
    for off, n in ((576, 32), (608 + 9216, 32), (9856 + 9216, 32), (19392, 1)):
        assert not p[off:off + n].any()
    params, out_scale, meta = LN.load_model()
    assert params.size == 19393 and out_scale > 0 and meta["samples"] > 0


def test_binding_rejects_views_the_c_side_cannot_address():
    # the C ABI reads N elements straight from the data pointer: a padded 2-D
    # view or a strided 1-D view must be refused before anything is called
    torch = pytest.importorskip("torch")
    A = S.Stencil(2, 4, 4, 1, (4.0, -1, -1, -1, -1, 0, 0))
    x = torch.zeros(16, dtype=torch.float64)
    padded = torch.zeros((4, 8), dtype=torch.float64)[:, :4]
    strided = torch.zeros(32, dtype=torch.float64)[::2]
    for bad in (padded, strided):
        with pytest.raises(ValueError, match="contiguous"):
            S.gmres_solve(A, bad, x, 2, 2, 1e-8)
    with pytest.raises(ValueError, match="float64"):
        S.gmres_solve(A, torch.zeros(16, dtype=torch.float32), x, 2, 2, 1e-8)
    # a block of columns may have a row stride, but not a short one
    with pytest.raises(ValueError, match="row stride"):
        S.kernel_gram(torch.zeros((2, 16), dtype=torch.float64).as_strided((2, 16), (8, 1)),
                      torch.zeros((1, 16), dtype=torch.float64))
