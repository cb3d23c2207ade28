"""GPU parity of the Hess-Smith (source + vortex) formulation against its
CPU oracle (oracle/panel_oracle_hs.c), through the C ABI.

The Hess-Smith system has 1/2 on the diagonal of its source block (a
second-kind equation), so it is far better conditioned than the
stream-function system: the FP64 bound 1e-10 and the FP32 + refinement
bound 1e-8 apply directly, on gamma (here the tangential surface speed),
Cp, Cl and Cl_p, with the oracle working on the GPU's own nodes.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

DEG = math.pi / 180.0
TOL = {0: 1e-10, 1: 1e-8}
HS = "hess_smith"
ENTRY_ULPS = 16


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _errors(got, ref, noff, aoff):
    Ns, Ks = np.diff(noff) - 1, np.diff(aoff)
    so = np.concatenate([[0], np.cumsum(Ns * Ks)])
    e = dict(cl=0.0, cl_p=0.0, cp=0.0, gamma=0.0)
    for b in range(len(Ns)):
        sa, ss = slice(aoff[b], aoff[b + 1]), slice(so[b], so[b + 1])
        e["cl"] = max(e["cl"], np.max(np.abs(got["cl"][sa] - ref["cl"][sa]) / np.maximum(1.0, np.abs(ref["cl"][sa]))))
        e["cl_p"] = max(e["cl_p"], np.max(np.abs(got["cl_p"][sa] - ref["cl_p"][sa]) /
                                          np.maximum(1.0, np.abs(ref["cl_p"][sa]))))
        e["cp"] = max(e["cp"], np.max(np.abs(got["cp"][ss] - ref["cp"][ss])) / max(1.0, np.max(np.abs(ref["cp"][ss]))))
        e["gamma"] = max(e["gamma"], np.max(np.abs(got["gamma"][ss] - ref["gamma"][ss])) /
                         max(1.0, np.max(np.abs(ref["gamma"][ss]))))
    return e


def _solve(w, precision, tiling=None, chord=None, vinf=1.0):
    import torch
    import paper_1511_02166_amd as P
    s = P.PanelSolver(w.node_offsets(), w.alpha_offsets(), precision, tiling=tiling,
                      formulation=P.PANEL_HESS_SMITH)
    xy = s.naca4(torch.as_tensor(w.mpt(), device="cuda"), w.closed_te)
    alpha = torch.as_tensor(w.alpha_flat(), device="cuda")
    ch = None if chord is None else torch.as_tensor(np.asarray(chord, dtype=np.float64), device="cuda")
    out = s.solve(xy, alpha, chord=ch, vinf=vinf)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    return s, xy, got


def _hs_entry_scale(P):
    """Size of the terms of each normal/tangential source entry,
    (|log r1^2| + |log r2^2| + 4 + 2 pi) / 4 pi (log of a rounded argument:
    a few eps absolute), so that a correct evaluation is within a few ulp of
    it; the vortex columns are row sums, bounded by the row's sum of scales."""
    P = np.asarray(P).reshape(-1, 2)
    m = 0.5 * (P[:-1] + P[1:])
    d1 = m[:, None, :] - P[None, :-1, :]
    d2 = m[:, None, :] - P[None, 1:, :]
    with np.errstate(divide="ignore"):
        l1 = np.abs(np.log((d1 ** 2).sum(-1)))
        l2 = np.abs(np.log((d2 ** 2).sum(-1)))
    T = (np.nan_to_num(l1, posinf=0) + np.nan_to_num(l2, posinf=0) + 4 + 2 * np.pi) / (4 * np.pi)
    return np.concatenate([T, T.sum(1, keepdims=True)], axis=1)


@pytest.mark.parametrize("n,K,vinf", [(64, 1, 1.0), (256, 3, 1.7), (1024, 2, 1.0)])
def test_hs_assembly_matches_oracle(n, K, vinf):
    import torch
    import paper_1511_02166_amd as P
    _say(f"Hess-Smith assembly: N={n}, K={K}, vinf={vinf}")
    rng = np.random.default_rng(n)
    nodes = [oracle.naca4(0.04, 0.35, 0.12, n), synth.joukowski_nodes(n, 0.25, complex(-0.03, 0.04))]
    xy_flat, noff = synth.pack_nodes(nodes)
    alphas = [rng.uniform(-4, 12, K) * DEG for _ in nodes]
    aoff = np.array([0, K, 2 * K], dtype=np.int32)
    s = P.PanelSolver(noff, aoff, P.PANEL_FP64, formulation=P.PANEL_HESS_SMITH)
    s.assemble(torch.as_tensor(xy_flat, device="cuda"), torch.as_tensor(np.concatenate(alphas), device="cuda"),
               vinf=vinf)
    torch.cuda.synchronize()
    eps = np.finfo(np.float64).eps
    for b in range(2):
        M, R = s.system(b)
        Tg = s.tangential(b)
        Mr, Rr, Tr = oracle.hs_assemble(nodes[b], alphas[b], vinf)
        S = _hs_entry_scale(nodes[b])
        rn = np.max(np.abs(M[:-1] - Mr[:-1]) / (eps * S))
        rt = np.max(np.abs(Tg - Tr) / (eps * S))
        # the Kutta row is the sum of two tangential rows
        rk = np.max(np.abs(M[-1] - Mr[-1]) / (eps * (S[0] + S[-1])))
        _say(f"  b={b}: normal {rn:.2f} ulp, tangential {rt:.2f} ulp, Kutta row {rk:.2f} ulp (bound {ENTRY_ULPS})")
        assert rn < ENTRY_ULPS and rt < ENTRY_ULPS and rk < 2 * ENTRY_ULPS
        assert np.max(np.abs(R - Rr)) < 8 * eps * vinf


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("tiling", [(320, 0, 0), (0, 0, 4), (320, 1, 4)], ids=["wave", "workgroup", "persistent"])
def test_hs_pipeline_matches_oracle(precision, tiling):
    _say(f"Hess-Smith pipeline parity, precision={precision}, tiling={tiling}")
    w = synth.random_workload(51, 40, n_choices=(16, 64, 130, 256, 300, 400, 512), k_max=3)
    chord = np.random.default_rng(51).uniform(0.5, 2.0, w.B)
    s, xy, got = _solve(w, precision, tiling=tiling, chord=chord, vinf=2.3)
    assert np.all(got["info"] == 0)
    ref = oracle.solve_batch(xy.cpu().numpy(), w.node_offsets(), w.alpha_flat(), w.alpha_offsets(), chord=chord,
                             vinf=2.3, formulation=HS)
    e = _errors(got, ref, w.node_offsets(), w.alpha_offsets())
    _say(f"  errors {e}")
    assert all(v < TOL[precision] for v in e.values()), e
    if precision == 1:
        it = s.refine_iterations()
        _say(f"  refinement sweeps {it.min()}..{it.max()}")
        assert it.max() <= 4


@pytest.mark.parametrize("precision", [0, 1])
def test_hs_ga_batch_2048(precision):
    # the GA-population batch in the Hess-Smith formulation, sampled parity
    _say(f"Hess-Smith, 2048 x N=256, precision={precision}")
    w = synth.workload("ga2048")
    s, xy, got = _solve(w, precision)
    assert np.all(got["info"] == 0)
    idx = np.array([0, 1, 511, 1024, 2047])
    ws = w.subset(idx)
    xh = xy.cpu().numpy()
    noff = w.node_offsets()
    xo = np.concatenate([xh[2 * noff[b]:2 * noff[b + 1]] for b in idx])
    ref = oracle.solve_batch(xo, ws.node_offsets(), ws.alpha_flat(), ws.alpha_offsets(), formulation=HS)
    sub = dict(cl=got["cl"][idx], cl_p=got["cl_p"][idx],
               cp=np.concatenate([got["cp"][256 * b:256 * (b + 1)] for b in idx]),
               gamma=np.concatenate([got["gamma"][256 * b:256 * (b + 1)] for b in idx]))
    e = _errors(sub, ref, ws.node_offsets(), ws.alpha_offsets())
    _say(f"  errors {e}")
    assert all(v < TOL[precision] for v in e.values()), e
    # Kutta condition on every airfoil: u_0 + u_{N-1} = 0
    u = got["gamma"].reshape(w.B, 256)
    k = np.max(np.abs(u[:, 0] + u[:, -1]) / np.max(np.abs(u), axis=1))
    _say(f"  Kutta residual {k:.1e}")
    assert k < (1e-12 if precision == 0 else 1e-9)


def test_hs_closed_forms_on_the_gpu():
    # cylinder: Cp = 1 - 4 sin^2 exactly at the midpoints; lifting cylinder
    # with the Kutta point at theta = 0: Cl -> 4 pi sin a (second order)
    import torch
    import paper_1511_02166_amd as P
    _say("Hess-Smith closed forms on the GPU")
    a = 5 * DEG
    nodes = [synth.circle_nodes(n, R=0.5) for n in (64, 128, 256)]
    xy_flat, noff = synth.pack_nodes(nodes)
    aoff = np.arange(4, dtype=np.int32) * 2
    s = P.PanelSolver(noff, aoff, P.PANEL_FP64, formulation=P.PANEL_HESS_SMITH)
    out = s.solve(torch.as_tensor(xy_flat, device="cuda"), torch.as_tensor(np.tile([0.0, a], 3), device="cuda"))
    torch.cuda.synchronize()
    cp = out["cp"].cpu().numpy()
    cl = out["cl"].cpu().numpy()
    so = 0
    errs = []
    for q, n in enumerate((64, 128, 256)):
        thm = 2 * np.pi * (np.arange(n) + 0.5) / n
        assert np.max(np.abs(cp[so:so + n] - (1 - 4 * np.sin(thm) ** 2))) < 1e-9
        so += 2 * n
        errs.append(abs(cl[2 * q + 1] - 4 * np.pi * np.sin(a)))
        assert abs(cl[2 * q]) < 1e-12
    _say(f"  lifting cylinder Cl errors {errs}")
    assert errs[2] < 2e-4 and errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_hs_graph_replay_noalloc_and_adjoint_refusal():
    import torch
    import paper_1511_02166_amd as P
    _say("Hess-Smith: graph replay, no-alloc entry point, adjoint refusal")
    w = synth.workload("ga2048", B=64)
    s, xy, got = _solve(w, 0)
    alpha = torch.as_tensor(w.alpha_flat(), device="cuda")
    eager = s.cl.clone()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            s.step(xy, alpha)
    torch.cuda.current_stream().wait_stream(side)
    for _ in range(3):
        s.cl.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(s.cl, eager)
    plan = P.Plan(w.node_offsets(), w.alpha_offsets(), P.PANEL_FP64, P.PANEL_HESS_SMITH)
    info = torch.zeros(w.B, dtype=torch.int32, device="cuda")
    cl = torch.empty(w.B, dtype=torch.float64, device="cuda")
    P.panel_solve_noalloc(plan, xy, alpha, None, 1.0, 1e-10, 10, info, None, None, cl, None)
    torch.cuda.synchronize()
    assert torch.equal(cl, eager) and int(info.abs().max()) == 0
    with pytest.raises(P.PanelError, match="stream-function"):
        s.adjoint(xy, torch.ones(w.B, dtype=torch.float64, device="cuda"))
