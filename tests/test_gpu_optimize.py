"""GBO / L-BFGS driven by the HIP path (needs a GPU): the periodic two-amplitude
identification recovers the exact discrete optimum."""
import numpy as np
import pytest

from paper_2609_31347_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_two_amplitude_identification_on_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import fourier as Fo
    from paper_2609_31347_amd import slbm as S
    from paper_2609_31347_amd.optimize import PAPER_BENCH1, gpu_objective, lbfgs
    n = 128
    modes = I.two_mode_basis(n)
    tgt = I.two_mode_target(n)
    ctx = S.solid_lbm_init(dict(nx=n, ny=n, dx=1 / n, E=1.0, nu=0.3, domain=0, target=tgt, control_kind=0,
                                n_modes=2, force_modes=modes, tol=1e-12))
    r = lbfgs(gpu_objective(ctx), np.array([0.1, 0.1]), **PAPER_BENCH1)
    # exact discrete optimum: d is linear in A; least squares over the two closed-form responses
    R = np.stack([Fo.steady_disp(m / n ** 2, 1.0, 0.3).ravel() for m in modes], 1)
    a_ex = np.linalg.lstsq(R, tgt.ravel(), rcond=None)[0]
    assert r.J < 1e-20
    assert np.abs(r.x - a_ex).max() < 1e-8
    assert r.steps <= 15
