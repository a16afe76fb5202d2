"""The learned denoiser against the plain estimator it corrects, on held-out
runs (the protocol of paper_1006_0720_amd/denoise_study.py, reduced): a
20k-triangle street canyon with the model coefficients frozen at one field,
so that every run samples the same particle process; the network is trained on the GPU by
the library's own kernels on 8 pairs of 10- and 200-particle-per-element
runs; 2 held-out source positions are scored against the ensemble mean of 3
independent 200-per-element runs each.  At the default tau = 3 with the
calibrated fallback, and without any fallback, the learned estimate's error
is below the plain 10-per-element estimator's, overall and for most of the 8
statistics; the plain estimator's error falls with the particle count."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1006_0720_amd import _lib
    return _lib


def test_learned_denoiser_gain_on_held_out_runs(L):
    from paper_1006_0720_amd.denoise_study import study
    from synth import configs as CF
    from synth import meshes as M

    mesh = M.canyon(20_000, 0.15, 0)

    def make(ppe, seed, src):
        return CF.canyon(mesh=mesh, ppe=ppe, seed=seed, src=src)

    res, _, _ = study(make, n_train=8, n_test=2, n_ref=3, steps_spin=40, n_snap=4, every=10, train_steps=1500,
                      batch=4096, eval_ppes=(20, 40), frozen=True,
                      log=lambda m: print(m, flush=True))
    Ep = res["E_plain"]
    lv = res["learned"]
    print({k: (round(v["E"], 4), round(v["ppe_eq"], 1), round(v["cost_ratio"], 2)) for k, v in lv.items()},
          {p: round(e, 4) for p, e in Ep.items()}, "kappa", np.round(res["kappa"], 2).tolist(), flush=True)
    assert Ep[10] > Ep[20] > Ep[40]
    for name in ("tau3_calibrated", "no_fallback"):
        assert lv[name]["E"] < Ep[10], name
        assert sum(r < 1.0 for r in lv[name]["per_statistic_over_plain"]) >= 6, name
    # the calibrated fallback accepts more of the network's corrections than the noise-only test
    assert lv["tau3_calibrated"]["rejected_fraction"] <= lv["tau3_noise"]["rejected_fraction"]
    assert all(k > 0.0 for k in res["kappa"])
