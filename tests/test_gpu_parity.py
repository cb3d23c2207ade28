"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle.

Tolerances (relative, as the lift and Cp cross zero):
  e_Cl = |Cl - Cl*| / max(1, |Cl*|),
  e_Cp = max_i |Cp_i - Cp*_i| / max(1, max_i |Cp*_i|)
with 1e-10 for the FP64 path and 1e-8 for FP32 factors + FP64 refinement,
and the same metric for the surface speed gamma.  Both sides always work on
the same node array: the GPU's own NACA nodes are copied back and handed to
the oracle (the NACA kernel has a parity test of its own).  Where a geometry
is conditioned badly enough that two correct FP64 solutions differ by more
than these tolerances, the bound becomes FLOOR_FACTOR times the floor
measured on that system (tests/_floor.py), which is logged beside the error.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from _floor import FLOOR_FACTOR, measured_floor

pytestmark = pytest.mark.gpu

DEG = math.pi / 180.0
TOL64 = 1e-10
TOL32R = 1e-8


def _torch():
    import torch
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _gpu_inputs(w, xy_flat=None):
    """Device inputs for a workload; nodes from the library's NACA kernel unless given."""
    import paper_1511_02166_amd as P
    torch = _torch()
    dev = "cuda"
    alpha = torch.as_tensor(w.alpha_flat(), device=dev)
    if xy_flat is None:
        s = P.PanelSolver(w.node_offsets(), w.alpha_offsets())
        xy = s.naca4(torch.as_tensor(w.mpt(), device=dev), w.closed_te)
    else:
        xy = torch.as_tensor(np.asarray(xy_flat, dtype=np.float64), device=dev)
    return xy, alpha


def _oracle(w, xy_flat, chord=None, vinf=1.0):
    """Oracle on exactly the nodes the GPU used."""
    return oracle.solve_batch(xy_flat, w.node_offsets(), w.alpha_flat(), w.alpha_offsets(), chord=chord,
                              vinf=vinf)


def _ok(e, tol):
    return all(e[k] < tol for k in ("cl", "cl_p", "cp", "gamma"))


def _assert_parity(got, ref, w, xy_flat, tol):
    """Per airfoil and quantity: error < tol, or, where the error is larger,
    < FLOOR_FACTOR x the floor measured on that airfoil's system (needed for
    the larger panel counts, whose FP64 floor reaches ~1e-10)."""
    noff, aoff = w.node_offsets(), w.alpha_offsets()
    Ns, Ks = np.diff(noff) - 1, np.diff(aoff)
    so = np.concatenate([[0], np.cumsum(Ns * Ks)])
    worst = 0.0
    for b in range(w.B):
        sa, ss = slice(aoff[b], aoff[b + 1]), slice(so[b], so[b + 1])
        e = dict(cl=np.max(np.abs(got["cl"][sa] - ref["cl"][sa]) / np.maximum(1.0, np.abs(ref["cl"][sa]))),
                 cl_p=np.max(np.abs(got["cl_p"][sa] - ref["cl_p"][sa]) / np.maximum(1.0, np.abs(ref["cl_p"][sa]))),
                 cp=np.max(np.abs(got["cp"][ss] - ref["cp"][ss])) / max(1.0, np.max(np.abs(ref["cp"][ss]))),
                 gamma=np.max(np.abs(got["gamma"][ss] - ref["gamma"][ss])) / max(1.0, np.max(np.abs(ref["gamma"][ss]))))
        worst = max(worst, max(e.values()))
        if _ok(e, tol):
            continue
        fl = measured_floor(xy_flat[2 * noff[b]:2 * noff[b + 1]], w.alpha[b])
        _say(f"  airfoil {b} N={Ns[b]}: " + " ".join(f"{q} {e[q]:.1e}/{fl[q]:.0e}" for q in e) + " (error/floor)")
        for q in e:
            assert e[q] < max(tol, FLOOR_FACTOR * fl[q]), (b, q, e[q], fl[q])
    return worst


def _errors(gpu, ref, w):
    """Per-airfoil worst relative errors of Cl and Cp (G10 reading)."""
    noff, aoff = w.node_offsets(), w.alpha_offsets()
    Ns, Ks = np.diff(noff) - 1, np.diff(aoff)
    so = np.concatenate([[0], np.cumsum(Ns * Ks)])
    e_cl = np.abs(gpu["cl"] - ref["cl"]) / np.maximum(1.0, np.abs(ref["cl"]))
    e_clp = np.abs(gpu["cl_p"] - ref["cl_p"]) / np.maximum(1.0, np.abs(ref["cl_p"]))
    e_cp = np.zeros(w.B)
    e_g = np.zeros(w.B)
    for b in range(w.B):
        sl = slice(so[b], so[b + 1])
        e_cp[b] = np.max(np.abs(gpu["cp"][sl] - ref["cp"][sl])) / max(1.0, np.max(np.abs(ref["cp"][sl])))
        e_g[b] = np.max(np.abs(gpu["gamma"][sl] - ref["gamma"][sl])) / max(1.0, np.max(np.abs(ref["gamma"][sl])))
    return dict(cl=e_cl.max(), cl_p=e_clp.max(), cp=e_cp.max(), gamma=e_g.max())


def _run(w, precision, xy_flat=None, refine_tol=1e-10, max_iter=10, wave_limit=None, chord=None, vinf=1.0,
         tiling=None):
    """GPU solve; returns (solver, outputs, the node array the GPU used)."""
    import paper_1511_02166_amd as P
    torch = _torch()
    xy, alpha = _gpu_inputs(w, xy_flat)
    s = P.PanelSolver(w.node_offsets(), w.alpha_offsets(), precision, wave_limit=wave_limit, tiling=tiling)
    ch = None if chord is None else torch.as_tensor(np.asarray(chord, dtype=np.float64), device="cuda")
    out = s.solve(xy, alpha, chord=ch, vinf=vinf, refine_tol=refine_tol, max_iter=max_iter)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    got["xy"] = xy.cpu().numpy()
    return s, got


def test_naca4_matches_oracle():
    _say("naca4 parity: uneven4096[:64]")
    w = synth.workload("uneven4096", B=64)
    xy, _ = _gpu_inputs(w)
    ref, _ = oracle.workload_nodes(w)
    got = xy.cpu().numpy()
    assert np.max(np.abs(got - ref)) < 4e-16
    # closed trailing edge: node N equals node 0 bitwise
    noff = w.node_offsets()
    for b in range(w.B):
        assert np.all(got[2 * noff[b]:2 * noff[b] + 2] == got[2 * noff[b + 1] - 2:2 * noff[b + 1]])


def _joukowski_workload(seed, B, n, alphas):
    xy_flat, noff = synth.joukowski_batch(seed, B, n)
    w = synth.Workload(f"jk{seed}", np.zeros(B), np.zeros(B), np.zeros(B),
                       (np.diff(noff) - 1).astype(np.int32), [np.asarray(a) for a in alphas])
    return w, xy_flat, noff


def _entry_magnitude(xyb):
    """Per-entry size of the terms the closed form adds up (numpy, [N, N]).

    Off the diagonal G_ji = -(1/4pi L)[(d1.h) log|d1|^2 - (d2.h) log|d2|^2
    - 2 L^2 + 2 (d1 x d2) theta] (d1 = m_j - P_i, d2 = m_j - P_{i+1}); with
    |d1 x d2| = L |eta| and |theta| <= pi, rounding in any correct evaluation
    of it is a few ulp of
      T_ji = (|d1||h| (|log|d1|^2| + 2) + |d2||h| (|log|d2|^2| + 2) + 2 L^2) / (4 pi L) + |eta|
    (the logarithm of an argument that carries its own rounding is off by a
    few eps in absolute terms, hence the + 2), and on the diagonal of
    (L/2pi)(1 + |log(L/2)|).  T does not grow with N."""
    P = np.asarray(xyb, dtype=np.float64).reshape(-1, 2)
    N = P.shape[0] - 1
    m = 0.5 * (P[:-1] + P[1:])
    h = P[1:] - P[:-1]
    L = np.hypot(h[:, 0], h[:, 1])
    d1 = m[:, None, :] - P[None, :-1, :]
    d2 = m[:, None, :] - P[None, 1:, :]
    n1 = np.hypot(d1[..., 0], d1[..., 1])
    n2 = np.hypot(d2[..., 0], d2[..., 1])
    with np.errstate(divide="ignore"):
        l1 = np.abs(np.log(n1 ** 2)) + 2.0
        l2 = np.abs(np.log(n2 ** 2)) + 2.0
    eta = np.abs(d1[..., 0] * h[None, :, 1] - d1[..., 1] * h[None, :, 0]) / L[None, :]
    T = (n1 * L[None, :] * l1 + n2 * L[None, :] * l2 + 2 * L[None, :] ** 2) / (4 * np.pi * L[None, :]) + eta
    d = np.arange(N)
    T[d, d] = L / (2 * np.pi) * (1 + np.abs(np.log(L / 2)))
    return T


# Largest difference allowed between the GPU's and the oracle's influence
# entries, in units of eps * T_ji: the GPU's logarithm is within 2 ulp, its
# arctangent within 3 ulp, and a closed form of ~12 operations adds a few more.
ENTRY_ULPS = 16


@pytest.mark.parametrize("seed,B,n,K", [(1, 4, 128, 2), (2, 2, 256, 2), (3, 2, 256, 16), (4, 2, 1024, 3)])
def test_assembly_entries_match_oracle(seed, B, n, K):
    _say(f"assembly parity: {B} joukowski sections, N={n}, K={K}, identical nodes")
    import paper_1511_02166_amd as P
    torch = _torch()
    rng = np.random.default_rng(seed)
    w, xy_flat, noff = _joukowski_workload(seed, B, n, [rng.uniform(-4, 12, K) * DEG for _ in range(B)])
    xy, alpha = _gpu_inputs(w, xy_flat)
    s = P.PanelSolver(noff, w.alpha_offsets())
    vinf = 1.0 if seed % 2 else 1.9
    s.assemble(xy, alpha, vinf=vinf)
    torch.cuda.synchronize()
    eps = np.finfo(np.float64).eps
    for b in range(B):
        M, rhs = s.system(b)
        xyb = xy_flat[2 * noff[b]:2 * noff[b + 1]]
        Mr, Rr = oracle.assemble(xyb, w.alpha[b], vinf)
        T = _entry_magnitude(xyb)
        ratio = np.max(np.abs(M[:-1, :-1] - Mr[:-1, :-1]) / (eps * T))
        _say(f"  b={b}: max |G - G_oracle| / (eps T) = {ratio:.2f} ulp (bound {ENTRY_ULPS})")
        assert ratio < ENTRY_ULPS
        assert np.all(M[:-1, -1] == -1.0) and np.all(M[-1] == Mr[-1])
        # right-hand sides: -vinf (m_y cos a - m_x sin a), a few ulp of vinf |m|
        mabs = np.max(np.abs(xyb))
        assert np.max(np.abs(rhs - Rr)) < 8 * eps * vinf * mabs


@pytest.mark.parametrize("name,B,wave_limit", [("naca128", 32, None), ("ga2048", 96, None), ("ga2048", 40, 0)])
def test_fp64_pipeline_matches_oracle(name, B, wave_limit):
    import paper_1511_02166_amd as P
    _say(f"fp64 pipeline parity: {name}[:{B}], wave_limit={wave_limit}")
    w = synth.workload(name, B=B)
    s, got = _run(w, P.PANEL_FP64, wave_limit=wave_limit)
    ref = _oracle(w, got["xy"])
    assert np.all(got["info"] == 0) and np.all(ref["info"] == 0)
    e = _errors(got, ref, w)
    _say(f"  errors {e}")
    assert _ok(e, TOL64), e


@pytest.mark.parametrize("name,B,wave_limit", [("naca128", 32, None), ("ga2048", 96, None), ("ga2048", 40, 0)])
def test_fp32_refined_pipeline_matches_oracle(name, B, wave_limit):
    import paper_1511_02166_amd as P
    _say(f"fp32+refine pipeline parity: {name}[:{B}], wave_limit={wave_limit}")
    w = synth.workload(name, B=B)
    s, got = _run(w, P.PANEL_FP32_REFINE, wave_limit=wave_limit)
    ref = _oracle(w, got["xy"])
    assert np.all(got["info"] == 0)
    e = _errors(got, ref, w)
    it = s.refine_iterations()
    _say(f"  errors {e}, sweeps min/max {it.min()}/{it.max()}")
    assert _ok(e, TOL32R), e
    assert it.min() >= 1 and it.max() <= 6


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("wave_limit,persistent", [(320, 1), (320, 0), (0, 1), (0, 0)])
def test_uneven_batch_matches_oracle(precision, wave_limit, persistent):
    # K = 1..4 per airfoil: odd counts exercise the refinement's single
    # right-hand-side tail in both kernel families, in one launch or separately
    _say(f"uneven batch parity, precision={precision}, wave_limit={wave_limit}, persistent={persistent}")
    w = synth.random_workload(11, 40, n_choices=(4, 6, 16, 30, 64, 96, 130, 250, 256, 300), k_max=4)
    s, got = _run(w, precision, tiling=(wave_limit, persistent, 4))
    ref = _oracle(w, got["xy"])
    assert np.all(got["info"] == 0)
    e = _errors(got, ref, w)
    tol = TOL64 if precision == 0 else TOL32R
    _say(f"  errors {e}")
    assert _ok(e, tol), e


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("wave_limit", [None, 0])
def test_max_angles_per_airfoil(precision, wave_limit):
    # K = 16 right-hand sides (the largest allowed) ride through the
    # factorisation as extra columns: the widest trailing blocks, including
    # n1 + K = 335 for the largest even panel count of the one-wavefront kernels.
    _say(f"K = 16 angles, precision={precision}, wave_limit={wave_limit}")
    w = synth.random_workload(17, 6, n_choices=(30, 64, 250, 300, 318), k_max=1)
    rng = np.random.default_rng(17)
    w = synth.Workload(w.name, w.m, w.p, w.t, np.array([30, 64, 250, 300, 316, 318], dtype=np.int32),
                       [rng.uniform(-4.0, 12.0, 16) * DEG for _ in range(6)], True)
    s, got = _run(w, precision, wave_limit=wave_limit)
    ref = _oracle(w, got["xy"])
    assert np.all(got["info"] == 0)
    e = _errors(got, ref, w)
    tol = TOL64 if precision == 0 else TOL32R
    _say(f"  errors {e}")
    assert _ok(e, tol), e


def test_closed_form_geometries_identical_inputs():
    # Cylinder and Joukowski nodes from the shared input generator, fed to both
    # sides.  The cusped Joukowski sections are much worse conditioned than the
    # NACA workloads, so each quantity's bound is max(base, FLOOR_FACTOR x the
    # floor measured on that system from the oracle alone).
    import paper_1511_02166_amd as P
    _say("cylinder / joukowski parity")
    nodes = [synth.circle_nodes(64), synth.joukowski_nodes(128), synth.circle_nodes(200, 0.3, 1.0, -2.0),
             synth.joukowski_nodes(256, 0.3, complex(-0.05, 0.06))]
    xy_flat, noff = synth.pack_nodes(nodes)
    al = [np.array([0.0, 5 * DEG]), np.array([4 * DEG]), np.array([-3 * DEG, 1 * DEG, 7 * DEG]),
          np.array([2 * DEG])]
    floors = [measured_floor(nd, a) for nd, a in zip(nodes, al)]
    w = synth.Workload("closed-form", np.zeros(4), np.zeros(4), np.zeros(4),
                       (np.diff(noff) - 1).astype(np.int32), al)
    aoff = w.alpha_offsets()
    so = np.concatenate([[0], np.cumsum((np.diff(noff) - 1) * np.diff(aoff))])
    for prec, base in ((P.PANEL_FP64, TOL64), (P.PANEL_FP32_REFINE, TOL32R)):
        s, got = _run(w, prec, xy_flat)
        ref = _oracle(w, xy_flat)
        for b in range(4):
            wb = w.subset([b])
            sl_a = slice(aoff[b], aoff[b + 1])
            sl_s = slice(so[b], so[b + 1])
            gb = {k: got[k][sl_a] for k in ("cl", "cl_p")}
            gb.update({k: got[k][sl_s] for k in ("cp", "gamma")})
            rb = {k: ref[k][sl_a] for k in ("cl", "cl_p")}
            rb.update({k: ref[k][sl_s] for k in ("cp", "gamma")})
            e = _errors(gb, rb, wb)
            for q in ("cl", "cl_p", "cp", "gamma"):
                tol = max(base, FLOOR_FACTOR * floors[b][q])
                _say(f"  prec {prec} geom {b} {q}: error {e[q]:.2e} floor {floors[b][q]:.2e} bound {tol:.2e}")
                assert e[q] < tol, (prec, b, q, e[q], floors[b][q])


def test_pivots_match_oracle_on_kutta_system():
    # The Kutta row wins the first pivot (|1| > |G_00|); the pivot choices are
    # far from ties here, so the sequences must agree exactly.
    import paper_1511_02166_amd as P
    torch = _torch()
    _say("pivot sequence parity")
    w, xy_flat, noff = _joukowski_workload(3, 3, 128, [[0.05]] * 3)
    xy, alpha = _gpu_inputs(w, xy_flat)
    s = P.PanelSolver(noff, w.alpha_offsets())
    s.solve(xy, alpha)
    torch.cuda.synchronize()
    for b in range(3):
        M, _ = oracle.assemble(xy_flat[2 * noff[b]:2 * noff[b + 1]], w.alpha[b])
        _, piv, _ = oracle.lu(M)
        assert piv[0] == 128
        assert np.array_equal(s.pivots(b), piv)


def test_info_codes_for_bad_geometry():
    import paper_1511_02166_amd as P
    _say("info codes: repeated node, NaN node")
    w, xy_flat, noff = _joukowski_workload(4, 3, 64, [[0.05]] * 3)
    xy_flat = xy_flat.copy()
    k = noff[1] + 5
    xy_flat[2 * (k + 1):2 * (k + 2)] = xy_flat[2 * k:2 * (k + 1)]   # zero-length panel in airfoil 1
    xy_flat[2 * (noff[2] + 9)] = np.nan                              # NaN in airfoil 2
    for prec in (P.PANEL_FP64, P.PANEL_FP32_REFINE):
        s, got = _run(w, prec, xy_flat)
        assert list(got["info"]) == [0, -1, -1]
        assert np.all(np.isfinite(got["cl"][:1])) and np.all(np.isnan(got["cl"][1:]))


def test_refinement_budget_exhausted_reports_minus_two():
    import paper_1511_02166_amd as P
    _say("refinement with max_iter=0 / unreachable tolerance")
    w = synth.workload("ga2048", B=4)
    _, got = _run(w, P.PANEL_FP32_REFINE, max_iter=0)
    assert np.all(got["info"] == -2)
    # one sweep cannot verify convergence: the FP32 start is far from the
    # FP64 floor and a 1e-30 correction target is unreachable
    _, got = _run(w, P.PANEL_FP32_REFINE, refine_tol=1e-30, max_iter=1)
    assert np.all(got["info"] == -2)
    assert np.all(np.isfinite(got["cl"]))


def test_graph_replay_matches_eager():
    import paper_1511_02166_amd as P
    torch = _torch()
    _say("hip graph capture/replay")
    w = synth.workload("ga2048", B=64)
    xy, alpha = _gpu_inputs(w)
    for prec in (P.PANEL_FP64, P.PANEL_FP32_REFINE):
        s = P.PanelSolver(w.node_offsets(), w.alpha_offsets(), prec)
        s.step(xy, alpha)
        torch.cuda.synchronize()
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


# Panel counts for the factor checks: full and partial 64-column super-panels
# and 16-column tails; 1..5 rows per thread (workgroup kernel, N > 319) and
# 1..5 rows per lane (wavefront kernel, N <= 319).
_SIZES_MIXED = [4, 30, 62, 64, 130, 190, 256, 300, 510, 700, 1024]
_SIZES_WAVE = [4, 15, 16, 17, 31, 62, 63, 64, 65, 100, 127, 128, 129, 191, 192, 193, 255, 256, 257, 300,
               318, 319]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("sizes,wave_limit", [(_SIZES_MIXED, None), (_SIZES_WAVE, None),
                                              (_SIZES_WAVE[::3], 0)],
                         ids=["mixed-kernels", "wavefront-kernel", "workgroup-kernel"])
def test_lu_factors_reproduce_matrix(precision, sizes, wave_limit):
    # Direct algebraic check of the stored factors: P A = L U (FP64 to 1e-13,
    # FP32 to its own rounding level), and the right-hand-side columns hold
    # L^{-1} P b.
    import paper_1511_02166_amd as P
    torch = _torch()
    _say(f"LU factor residual, precision={precision}, wave_limit={wave_limit}, N={sizes}")
    xy_flat, noff = synth.joukowski_batch(31, len(sizes), sizes)
    aoff = np.arange(len(sizes) + 1, dtype=np.int32) * 2
    s = P.PanelSolver(noff, aoff, precision, wave_limit=wave_limit)
    xy = torch.as_tensor(xy_flat, device="cuda")
    al = torch.as_tensor(np.tile([0.03, 0.1], len(sizes)), device="cuda")
    s.assemble(xy, al)
    torch.cuda.synchronize()
    mats = [s.system(b) for b in range(len(sizes))]
    s.factor_solve()
    torch.cuda.synchronize()
    assert np.all(s.info.cpu().numpy() == 0)
    tol = 1e-13 if precision == 0 else 2e-6
    for b, N in enumerate(sizes):
        A, R = mats[b]
        LU, Y = s.system(b, "a64" if precision == 0 else "a32")
        LU = LU.astype(np.float64)
        piv = s.pivots(b)
        n = N + 1
        PA = A.copy()
        PR = R.copy()
        for i in range(n):
            p = piv[i]
            assert i <= p < n
            PA[[i, p]] = PA[[p, i]]
            PR[:, [i, p]] = PR[:, [p, i]]
        Lm = np.tril(LU, -1) + np.eye(n)
        Um = np.triu(LU)
        res = np.max(np.abs(PA - Lm @ Um)) / np.max(np.abs(A))
        _say(f"  N={N}: |PA-LU|/|A| = {res:.2e}")
        assert res < tol * n, (N, res)
        ry = np.max(np.abs(Lm @ Y.T.astype(np.float64) - PR.T)) / np.max(np.abs(R))
        assert ry < tol * n, (N, ry)


def test_autotune_picks_a_tiling_and_keeps_results(tmp_path):
    # the measured tiling changes which kernels run, not the answer; the
    # table file makes the next search for the same layout a lookup
    import paper_1511_02166_amd as P
    torch = _torch()
    w = synth.random_workload(43, 96, n_choices=(64, 128, 256, 300, 400, 510), k_max=2)
    _say("autotune of the tiling, 96 mixed sections (N 64..510), both precisions")
    xy, alpha = _gpu_inputs(w)
    ref = _oracle(w, xy.cpu().numpy())
    table = P.TileTable(str(tmp_path / "tiles.json"))
    for prec, tol in ((P.PANEL_FP64, TOL64), (P.PANEL_FP32_REFINE, TOL32R)):
        s = P.PanelSolver(w.node_offsets(), w.alpha_offsets(), prec)
        cands = s.tiling_candidates()
        times = s.autotune(xy, alpha, table=table)
        best = min(times, key=times.get)
        _say(f"  precision {prec}: {len(cands)} candidates, best {best} at {times[best]:.3f} ms")
        assert set(times) == set(cands) and len(cands) > 4
        t = s.tiling
        assert (t["wave_max_n1"], t["persistent"], t["wg_waves"]) == best
        out = s.solve(xy, alpha)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        assert np.all(got["info"] == 0)
        _assert_parity(got, ref, w, xy.cpu().numpy(), tol)
        # a second solver with the same layout takes the stored entry
        s2 = P.PanelSolver(w.node_offsets(), w.alpha_offsets(), prec)
        assert s2.autotune(xy, alpha, table=P.TileTable(str(tmp_path / "tiles.json"))) == times
        t2 = s2.tiling
        assert (t2["wave_max_n1"], t2["persistent"], t2["wg_waves"]) == best


@pytest.mark.parametrize("precision", [0, 1])
def test_persistent_launch_matches_separate_launches(precision):
    # The persistent kernel runs the same per-airfoil arithmetic as the
    # separate kernels, only scheduled from one queue: identical results,
    # also on a second and third call (its queue counters reset themselves)
    # and with the wave limit moved so that the workgroup path takes a share.
    import paper_1511_02166_amd as P
    torch = _torch()
    w = synth.random_workload(47, 70, n_choices=(4, 30, 64, 128, 250, 300, 318, 320, 400, 510, 640, 766), k_max=3)
    _say(f"persistent vs separate launches, precision={precision}")
    xy, alpha = _gpu_inputs(w)
    ref = _oracle(w, xy.cpu().numpy())
    tol = TOL64 if precision == 0 else TOL32R
    for wl in (320, 192):
        outs = []
        for tiling in ((wl, 1, 4), (wl, 0, 4), (wl, 0, 8)):
            s = P.PanelSolver(w.node_offsets(), w.alpha_offsets(), precision, tiling=tiling)
            for rep in range(3):
                out = s.solve(xy, alpha)
                torch.cuda.synchronize()
                got = {k: v.cpu().numpy() for k, v in out.items()}
                assert np.all(got["info"] == 0), (tiling, rep, got["info"])
                worst = _assert_parity(got, ref, w, xy.cpu().numpy(), tol)
            outs.append(got)
            _say(f"  tiling {tiling}: worst error {worst:.2e}")
        # four-wavefront workgroups, one launch or two: the same arithmetic
        for k in ("gamma", "cp", "cl", "cl_p"):
            assert np.array_equal(outs[0][k], outs[1][k]), (wl, k)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("wave_limit", [None, 0])
def test_chord_and_freestream_speed(precision, wave_limit):
    # Per-airfoil chords and vinf != 1 reach the right-hand side (vinf), Cp
    # (gamma / vinf), both lift coefficients (1 / (vinf c), 1 / c) and the
    # adjoint's seed: the whole path against the oracle with the same values.
    import paper_1511_02166_amd as P
    torch = _torch()
    _say(f"chord / vinf != 1, precision={precision}, wave_limit={wave_limit}")
    w = synth.random_workload(29, 12, n_choices=(16, 64, 130, 256, 300), k_max=3)
    rng = np.random.default_rng(29)
    chord = rng.uniform(0.4, 2.5, w.B)
    vinf = 3.7
    s, got = _run(w, precision, wave_limit=wave_limit, chord=chord, vinf=vinf)
    ref = _oracle(w, got["xy"], chord=chord, vinf=vinf)
    assert np.all(got["info"] == 0)
    e = _errors(got, ref, w)
    tol = TOL64 if precision == 0 else TOL32R
    _say(f"  errors {e}")
    assert _ok(e, tol), e
    # gamma itself scales with vinf: compare it against the oracle directly
    rel = np.max(np.abs(got["gamma"] - ref["gamma"])) / np.max(np.abs(ref["gamma"]))
    assert rel < tol, rel
    # adjoint with the same chords and speed
    noff, aoff = w.node_offsets(), w.alpha_offsets()
    dcl = rng.standard_normal(int(aoff[-1]))
    xy = torch.as_tensor(got["xy"], device="cuda")
    g = s.adjoint(xy, torch.as_tensor(dcl, device="cuda")).cpu().numpy()
    for b in range(w.B):
        xyb = got["xy"][2 * noff[b]:2 * noff[b + 1]]
        gr = sum(dcl[aoff[b] + k] * oracle.cl_gradient(xyb, a, vinf=vinf, chord=chord[b])
                 for k, a in enumerate(w.alpha[b]))
        gb = g[2 * noff[b]:2 * noff[b + 1]].reshape(-1, 2)
        eg = np.max(np.abs(gb - gr)) / np.max(np.abs(gr))
        assert eg < (1e-9 if precision == 0 else 1e-8), (b, eg)


@pytest.mark.parametrize("precision", [0, 1])
def test_heavy_pivoting_dense_systems(precision):
    # Panel systems hardly pivot (the Kutta row swaps twice), so the row moves
    # of the wavefront LU are exercised here on dense systems written over the
    # assembled ones in the workspace (its documented layout): Gaussian entries
    # pivot at nearly every step (up to 32 rows moved per 16-column panel), a
    # Gaussian matrix plus a diagonal shift of 6 at some (0, 2, 4 and 17 to 22
    # rows per panel), one shifted by 40 at none.  Checks P A = L U with every
    # multiplier |l| <= 1 (the partial-pivoting property) and the solutions
    # against the oracle's LU, within 64 eps times the condition number.
    import paper_1511_02166_amd as P
    torch = _torch()
    sizes = [255, 130, 200]
    _say(f"heavy pivoting, precision={precision}, N={sizes}")
    xy_flat, noff = synth.joukowski_batch(5, len(sizes), sizes)
    aoff = np.arange(len(sizes) + 1, dtype=np.int32) * 2
    s = P.PanelSolver(noff, aoff, precision)
    xy = torch.as_tensor(xy_flat, device="cuda")
    s.assemble(xy, torch.as_tensor(np.tile([0.02, 0.15], len(sizes)), device="cuda"))
    torch.cuda.synchronize()
    rng = np.random.default_rng(71)
    mats = []
    for b, N in enumerate(sizes):
        n = N + 1
        d = s.plan.layout(b)
        ld, K = d["ld"], d["K"]
        A = rng.standard_normal((n, n)) + (0.0, 6.0, 40.0)[b] * np.eye(n)
        R = rng.standard_normal((K, n))
        full = np.zeros((n + K, ld))
        full[:n, :n] = A.T          # column-major: row j of `full` is column j
        full[n:, :n] = R
        s.ws[d["a64"]:d["a64"] + 8 * full.size].copy_(
            torch.as_tensor(full.reshape(-1)).view(torch.uint8))
        if precision == 1:
            s.ws[d["a32"]:d["a32"] + 4 * full.size].copy_(
                torch.as_tensor(full.reshape(-1).astype(np.float32)).view(torch.uint8))
        mats.append((A, R))
    s.factor_solve()
    torch.cuda.synchronize()
    assert np.all(s.info.cpu().numpy() == 0)
    moved = []
    for b, N in enumerate(sizes):
        n = N + 1
        A, R = mats[b]
        d = s.plan.layout(b)
        LU, _ = s.system(b, "a64" if precision == 0 else "a32")
        LU = LU.astype(np.float64)
        piv = s.pivots(b)
        PA = A.copy()
        for i in range(n):
            assert i <= piv[i] < n
            PA[[i, piv[i]]] = PA[[piv[i], i]]
        Lm = np.tril(LU, -1) + np.eye(n)
        tol = 1e-13 if precision == 0 else 2e-6
        res = np.max(np.abs(PA - Lm @ np.triu(LU))) / np.max(np.abs(A))
        assert res < tol * n, (b, res)
        assert np.max(np.abs(np.tril(LU, -1))) <= 1.0 + 1e-12, b
        moved.append(int(np.sum(piv != np.arange(n))))
        X = s.ws[d["x"]:d["x"] + 8 * d["K"] * n].view(torch.float64).cpu().numpy().reshape(d["K"], n)
        oLU, opiv, oinfo = oracle.lu(A)
        assert oinfo == 0
        Xo = oracle.lu_solve(oLU, opiv, R)
        err = np.max(np.abs(X - Xo)) / np.max(np.abs(Xo))
        kappa = np.linalg.cond(A, np.inf)
        bound = max(1e-11 if precision == 0 else 1e-9, 64 * np.finfo(np.float64).eps * kappa)
        _say(f"  N={N}: rows moved {moved[-1]}, |PA-LU|/|A| {res:.1e}, solution error {err:.1e}"
             f" (bound {bound:.1e})")
        assert err < bound, (b, err, bound)
    assert moved[0] > 0.8 * sizes[0] and 0 < moved[1] < moved[0] and moved[2] == 0


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("wave_limit", [None, 0])
def test_exact_zero_pivot_reports_column(precision, wave_limit):
    # An exactly singular system: the assembled matrix of airfoil 1 with one
    # column zeroed in the workspace (its documented layout), so the column
    # stays exactly zero through every update.  LAPACK's getrf convention:
    # info = that column (1-based), elimination continues; this airfoil's
    # outputs are NaN, the others are untouched.  The oracle, pinned to the
    # same convention on the CPU, factors the same matrix.
    import paper_1511_02166_amd as P
    torch = _torch()
    _say(f"exact zero pivot, precision={precision}, wave_limit={wave_limit}")
    w, xy_flat, noff = _joukowski_workload(3, 3, 128, [[0.05]] * 3)
    xy, alpha = _gpu_inputs(w, xy_flat)
    for col in (5, 70, 128):
        s = P.PanelSolver(noff, w.alpha_offsets(), precision, wave_limit=wave_limit)
        s.assemble(xy, alpha)
        torch.cuda.synchronize()
        M, _ = s.system(1)
        d = s.plan.layout(1)
        ld = d["ld"]
        s.ws[d["a64"] + 8 * col * ld:d["a64"] + 8 * (col + 1) * ld].zero_()
        if precision == 1:
            s.ws[d["a32"] + 4 * col * ld:d["a32"] + 4 * (col + 1) * ld].zero_()
        s.factor_solve()
        s.forces()
        torch.cuda.synchronize()
        info = s.info.cpu().numpy()
        Mz = M.copy()
        Mz[:, col] = 0.0
        _, piv, oinfo = oracle.lu(Mz)
        _say(f"  column {col}: info {list(info)}, oracle info {oinfo}")
        assert oinfo == col + 1
        assert info[1] == oinfo and info[0] == 0 and info[2] == 0
        if precision == 0:
            assert np.array_equal(s.pivots(1), piv)
        cl = s.cl.cpu().numpy()
        assert np.isnan(cl[1]) and np.all(np.isfinite(cl[[0, 2]]))
        ref = _oracle(w, xy_flat)
        assert np.max(np.abs(cl[[0, 2]] - ref["cl"][[0, 2]])) < (TOL64 if precision == 0 else TOL32R)
        dxy = s.adjoint(xy, torch.ones(3, dtype=torch.float64, device="cuda")).cpu().numpy()
        assert np.all(np.isnan(dxy[2 * noff[1]:2 * noff[2]]))
        assert np.all(np.isfinite(dxy[:2 * noff[1]])) and np.all(np.isfinite(dxy[2 * noff[2]:]))
