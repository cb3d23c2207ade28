"""Accuracy of the library's own FP64 log and atan2 (used by the assembly and
adjoint kernels) against the host libm, in units in the last place."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _ulp_err(got, ref):
    return np.abs(got - ref) / np.spacing(np.maximum(np.abs(ref), np.finfo(float).tiny))


def test_log_and_atan2_ulp_error():
    import torch
    import paper_1511_02166_amd as P
    print("math accuracy: 2e6 random inputs", flush=True)
    rng = np.random.default_rng(5)
    n = 2_000_000
    # squared distances between control points and nodes span ~1e-12..20
    x = np.exp(rng.uniform(np.log(1e-14), np.log(1e3), n))
    x[: n // 10] = 1.0 + rng.uniform(-1e-4, 1e-4, n // 10)
    y = rng.standard_normal(n) * np.exp(rng.uniform(-25, 3, n))
    xa = rng.standard_normal(n) * np.exp(rng.uniform(-25, 3, n))
    lg = torch.empty(n, dtype=torch.float64, device="cuda")
    at = torch.empty(n, dtype=torch.float64, device="cuda")
    P.panel_math_eval(torch.as_tensor(x, device="cuda"), torch.as_tensor(y, device="cuda"), lg, None)
    P.panel_math_eval(torch.as_tensor(xa, device="cuda"), torch.as_tensor(y, device="cuda"), None, at)
    torch.cuda.synchronize()
    e_log = _ulp_err(lg.cpu().numpy(), np.log(x))
    e_at = _ulp_err(at.cpu().numpy(), np.arctan2(y, xa))
    print(f"  log max {e_log.max():.2f} ulp (mean {e_log.mean():.3f}); "
          f"atan2 max {e_at.max():.2f} ulp (mean {e_at.mean():.3f})", flush=True)
    assert e_log.max() <= 2.0
    assert e_at.max() <= 3.0
    # exact special values the kernels rely on
    sv = torch.tensor([1.0, 2.0, 0.5], dtype=torch.float64, device="cuda")
    lo = torch.empty(3, dtype=torch.float64, device="cuda")
    P.panel_math_eval(sv, sv, lo, None)
    assert lo[0].item() == 0.0
