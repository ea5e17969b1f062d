"""What the trained initial-guess network buys the solver (GPU), judged by
the solver's true residual.  On held-out 256^2 diffusion problems every solve
converges to 1e-8 in the true residual -- from x0 = 0, from x0 = 0 followed by
the same Jacobi sweeps and fallback rule the guess goes through (the ablation
that leaves the network out), from the guess with the fallback rule and from
the raw guess -- and where the fallback fires the solve is exactly the x0 = 0
solve.  The guess with the fallback rule must need fewer s-blocks on average
than both x0 = 0 and the sweeps-only ablation: the gain is the network's, not
the smoothing's."""
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


def test_trained_guess_beats_zero_and_sweeps_only_on_held_out_problems():
    S.load()
    params, out_scale, meta = LN.load_model()
    print(f"model trained on {meta.get('samples')} solved samples", flush=True)
    ds = LN.generate(24, 7000, nstreams=4, graph=True)
    res = LN.evaluate(params, out_scale, ds, meta["coarsen"], meta["sweeps"], nstreams=4,
                      graph=True)
    for mode in LN.MODES:
        assert np.all(res[mode]["status"] == S.OK), mode
    b = {m: res[m]["blocks"] for m in LN.MODES}
    print("mean blocks " + ", ".join(f"{m} {b[m].mean():.1f}" for m in LN.MODES)
          + f"; fallback {res['fallback'].mean():.2f}", flush=True)
    # where the fallback fired the solve starts from 0 and matches x0 = 0 exactly
    fb = res["fallback"]
    np.testing.assert_array_equal(b["cnn"][fb], b["zero"][fb])
    fbj = res["fallback_jacobi"]
    np.testing.assert_array_equal(b["jacobi"][fbj], b["zero"][fbj])
    assert b["cnn"].mean() < b["zero"].mean()
    assert b["cnn"].mean() < b["jacobi"].mean()
