"""What the trained initial-guess network buys the solver (GPU), judged by
the solver's true residual.  On held-out 256^2 diffusion problems every solve
(from x0 = 0, from the guess with the fallback rule, from the raw guess)
converges to 1e-8 in the true residual, and where the fallback fires the solve
is exactly the x0 = 0 solve.  The block counts of the three are printed: the
size (and sign) of the raw guess's gain is parity-unpinned -- no reference
value exists for it -- and is reported by the benchmark's learned workload."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2001_04886_amd import learn as LN
from paper_2001_04886_amd import sstep as S

pytestmark = pytest.mark.gpu


def test_committed_model_exists():
    assert os.path.exists(LN.DEFAULT_MODEL)
    params, out_scale, meta = LN.load_model()
    assert params.size == S.cnn_param_count() and out_scale > 0.0


def test_trained_guess_gain_on_held_out_problems():
    S.load()
    params, out_scale, meta = LN.load_model()
    ds = LN.generate(4, 7000, nstreams=1)
    res = LN.evaluate(params, out_scale, ds, meta["coarsen"], meta["sweeps"])
    for mode in ("zero", "cnn", "cnn_nofallback"):
        assert np.all(res[mode]["status"] == S.OK), mode
    zero, raw = res["zero"]["blocks"], res["cnn_nofallback"]["blocks"]
    print(f"blocks x0=0 {zero.tolist()}  network guess {raw.tolist()}  "
          f"fallback {res['fallback'].tolist()}")
    fb = res["fallback"]
    # where the fallback fired the solve starts from 0 and matches x0 = 0 exactly
    np.testing.assert_array_equal(res["cnn"]["blocks"][fb], zero[fb])
