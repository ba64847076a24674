"""The two FP64 reciprocals the kernels use in place of a divide, checked on the device against
the correctly rounded 1/x of the host.

- The residual sweep's law takes 1/(1 + s^2) as the hardware estimate refined by one Newton
  step: the step squares the estimate's relative error, so the result must be within 1e-14
  relative for every x >= 1 of the normal range (the law's value then carries at most that
  relative error in its s-dependent part, far below the 1e-12 operator parity).
- The V-cycle's Jacobi inverse takes two Newton steps: within 2 units in the last place for
  every normal x > 0 whose reciprocal is normal.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2502_21013_amd as P
    P.library()
    return P


def _rel(y, x):
    exact = 1.0 / x                      # correctly rounded (IEEE division)
    return np.abs(y - exact) / exact


def test_law_reciprocal_one_newton_step(gpu, P):
    rng = np.random.default_rng(7)
    x = np.concatenate([
        [1.0, np.nextafter(1.0, 2.0), 2.0, 3.0, 1e300],
        1.0 + np.logspace(-20, 300, 400001),          # 1 + s^2 over the whole range
        rng.uniform(1.0, 2.0, 200000),                # every mantissa pattern class
        np.ldexp(1.0, np.arange(0, 997)),             # powers of two
        np.ldexp(1.0, np.arange(0, 997)) * (2.0 - 2.0 ** -52),
    ])
    y1, _ = P.device_reciprocals(torch.from_numpy(x).to(gpu))
    err = _rel(y1.cpu().numpy(), x)
    worst = float(err.max())
    print(f"one-step reciprocal: max relative error {worst:.3e} over {x.size} points", flush=True)
    assert np.isfinite(err).all()
    assert worst <= 1e-14


def test_jacobi_reciprocal_two_newton_steps(gpu, P):
    rng = np.random.default_rng(8)
    x = np.concatenate([
        np.logspace(-300, 300, 400001),
        rng.uniform(0.5, 1.0, 200000),
        np.ldexp(1.0, np.arange(-1000, 1000)),
        np.ldexp(1.0, np.arange(-1000, 1000)) * (2.0 - 2.0 ** -52),
    ])
    _, y2 = P.device_reciprocals(torch.from_numpy(x).to(gpu))
    y2 = y2.cpu().numpy()
    ulp = np.spacing(1.0 / x)
    err_ulp = np.abs(y2 - 1.0 / x) / ulp
    worst = float(err_ulp.max())
    print(f"two-step reciprocal: max error {worst:.2f} ulp over {x.size} points", flush=True)
    assert np.isfinite(err_ulp).all()
    assert worst <= 2.0


def test_reciprocal_entry_point_validation(gpu, P):
    lib = P.library()
    assert lib.pt_device_reciprocals(None, None, 0, None) == 0
    assert lib.pt_device_reciprocals(None, None, -1, None) != 0
    assert lib.pt_device_reciprocals(None, None, 4, None) != 0
