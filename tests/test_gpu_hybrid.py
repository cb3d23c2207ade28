"""The paper's hybrid scheme (device assembly, host LAPACK solves in
slices), kept as an ablation: its lift must match the all-device path and
the oracle, for any slice count, in FP64 (and to single precision for the
FP32 copy).
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("slices", [1, 3, 7])
def test_hybrid_matches_all_device_and_oracle(slices):
    import torch
    import paper_1511_02166_amd as P
    from paper_1511_02166_amd.hybrid import HybridSolver
    _say(f"hybrid, {slices} slices")
    w = synth.random_workload(71, 40, n_choices=(64, 128, 200, 256), k_max=3)
    noff, aoff = w.node_offsets(), w.alpha_offsets()
    s = P.PanelSolver(noff, aoff, P.PANEL_FP64)
    xy = s.naca4(torch.as_tensor(w.mpt(), device="cuda"), True)
    alpha = torch.as_tensor(w.alpha_flat(), device="cuda")
    chord = torch.as_tensor(np.random.default_rng(1).uniform(0.5, 2.0, w.B), device="cuda")
    s.solve(xy, alpha, chord=chord, vinf=1.3)
    dev_cl = s.cl.cpu().numpy()
    h = HybridSolver(noff, aoff, slices, threads=8)
    cl, t = h.step(xy, alpha, chord=chord, vinf=1.3)
    h.close()
    e = np.max(np.abs(cl - dev_cl) / np.maximum(1.0, np.abs(dev_cl)))
    ref = oracle.solve_batch(xy.cpu().numpy(), noff, w.alpha_flat(), aoff, chord=chord.cpu().numpy(), vinf=1.3)
    eo = np.max(np.abs(cl - ref["cl"]) / np.maximum(1.0, np.abs(ref["cl"])))
    _say(f"  vs all-device {e:.1e}, vs oracle {eo:.1e}; W {t['W']:.3f} s, L {t['L']:.3f} s, "
         f"{t['bytes'] / 1e6:.0f} MB over the bus")
    assert e < 1e-10 and eo < 1e-10


def test_hybrid_fp32_copy():
    import torch
    import paper_1511_02166_amd as P
    from paper_1511_02166_amd.hybrid import HybridSolver
    _say("hybrid, FP32 systems")
    w = synth.workload("ga2048", B=48)
    noff, aoff = w.node_offsets(), w.alpha_offsets()
    s = P.PanelSolver(noff, aoff, P.PANEL_FP64)
    xy = s.naca4(torch.as_tensor(w.mpt(), device="cuda"), True)
    alpha = torch.as_tensor(w.alpha_flat(), device="cuda")
    s.solve(xy, alpha)
    h = HybridSolver(noff, aoff, 4, threads=8, precision=P.PANEL_FP32_REFINE)
    cl, t = h.step(xy, alpha)
    h.close()
    e = np.max(np.abs(cl - s.cl.cpu().numpy()))
    _say(f"  FP32 solve vs FP64 {e:.1e}")
    # single-precision LU of a system with condition ~1e6: a few 1e-4 at most
    assert e < 5e-3
