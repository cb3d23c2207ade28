"""The no-allocation entry point (panel_solve_noalloc) against the
caller-owned workspace path, through the C ABI.

Two calls in a row on the library's static scratch, the second with a
smaller, different batch (uneven N and K, the other precision), must each
reproduce what panel_workspace_init -> assemble -> factor_solve -> forces
give on a workspace of the caller's; a plan too large for the scratch is
refused before any HIP call.
"""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-8}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(w, precision, chord=None, vinf=1.0):
    import torch
    import paper_1511_02166_amd as P
    dev = "cuda"
    noff, aoff = w.node_offsets(), w.alpha_offsets()
    alpha = torch.as_tensor(w.alpha_flat(), device=dev)
    ref = P.PanelSolver(noff, aoff, precision)
    xy = ref.naca4(torch.as_tensor(w.mpt(), device=dev), True)
    ch = None if chord is None else torch.as_tensor(chord, device=dev)
    ref.solve(xy, alpha, chord=ch, vinf=vinf)
    plan = P.Plan(noff, aoff, precision)
    assert plan.workspace_size() <= P.PANEL_NOALLOC_MAX_BYTES
    f64 = dict(dtype=torch.float64, device=dev)
    info = torch.full((w.B,), 99, dtype=torch.int32, device=dev)
    gamma = torch.full((plan.n_out,), float("nan"), **f64)
    cp = torch.full((plan.n_out,), float("nan"), **f64)
    cl = torch.full((plan.n_alpha,), float("nan"), **f64)
    cl_p = torch.full((plan.n_alpha,), float("nan"), **f64)
    P.panel_solve_noalloc(plan, xy, alpha, ch, vinf, 1e-10, 10, info, gamma, cp, cl, cl_p)
    torch.cuda.synchronize()
    got = dict(info=info, gamma=gamma, cp=cp, cl=cl, cl_p=cl_p)
    want = dict(info=ref.info, gamma=ref.gamma, cp=ref.cp, cl=ref.cl, cl_p=ref.cl_p)
    assert torch.equal(got["info"], want["info"]) and int(info.abs().max()) == 0
    for k in ("gamma", "cp", "cl", "cl_p"):
        g, r = got[k].cpu().numpy(), want[k].cpu().numpy()
        e = np.max(np.abs(g - r)) / max(1.0, np.max(np.abs(r)))
        _say(f"  {k}: max rel diff {e:.2e}{' (bitwise equal)' if np.array_equal(g, r) else ''}")
        assert e < TOL[precision], (k, e)
    return plan


def test_noalloc_matches_workspace_path_twice():
    import paper_1511_02166_amd as P
    _say("no-alloc call 1: ga2048[:160], FP64")
    w1 = synth.workload("ga2048", B=160)
    _case(w1, P.PANEL_FP64)
    _say("no-alloc call 2 (smaller): 40 mixed sections N=16..300, K=1..3, FP32 + refinement, chords, vinf=2")
    w2 = synth.random_workload(37, 40, n_choices=(16, 64, 130, 256, 300), k_max=3)
    chord = np.random.default_rng(37).uniform(0.5, 2.0, w2.B)
    _case(w2, P.PANEL_FP32_REFINE, chord=chord, vinf=2.0)


def test_noalloc_refuses_a_plan_beyond_the_scratch():
    import torch
    import paper_1511_02166_amd as P
    w = synth.workload("ga2048", B=1024)
    plan = P.Plan(w.node_offsets(), w.alpha_offsets(), P.PANEL_FP64)
    assert plan.workspace_size() > P.PANEL_NOALLOC_MAX_BYTES
    t = torch.zeros(2 * plan.n_nodes, dtype=torch.float64, device="cuda")
    i = torch.zeros(w.B, dtype=torch.int32, device="cuda")
    with pytest.raises(P.PanelError, match="static scratch"):
        P.panel_solve_noalloc(plan, t, t, None, 1.0, 1e-10, 10, i, None, None, t, None)
