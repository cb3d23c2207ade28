"""GPU parity of the viscous correction (Thwaites' method, panel_thwaites)
against the CPU oracle (oracle/panel_oracle_bl.c), through the C ABI.

The boundary layer is run on the GPU's own surface speeds on both sides, so
the comparison isolates this step: cd and ld must agree to a few ulp of the
sums involved (the GPU's running integral is a blocked scan, the oracle's a
left-to-right loop), the separation panels exactly.  End to end (oracle
solve + oracle layer) they must agree to the solve's tolerance.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
DEG = math.pi / 180.0


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(w, formulation, re, precision=0):
    import torch
    import paper_1511_02166_amd as P
    s = P.PanelSolver(w.node_offsets(), w.alpha_offsets(), precision, formulation=formulation)
    xy = s.naca4(torch.as_tensor(w.mpt(), device="cuda"), True)
    s.solve(xy, torch.as_tensor(w.alpha_flat(), device="cuda"))
    bl = s.viscous(re)
    torch.cuda.synchronize()
    return (xy.cpu().numpy(), s.gamma.cpu().numpy(), s.cl.cpu().numpy(),
            {k: v.cpu().numpy() for k, v in bl.items()})


def _oracle_layer(w, xy, gamma, cl, re):
    noff, aoff = w.node_offsets(), w.alpha_offsets()
    Ns, Ks = np.diff(noff) - 1, np.diff(aoff)
    so = np.concatenate([[0], np.cumsum(Ns * Ks)])
    cd, ld, sep = [], [], []
    for b in range(w.B):
        r = oracle.thwaites(xy[2 * noff[b]:2 * noff[b + 1]], w.alpha[b], gamma[so[b]:so[b + 1]],
                            cl[aoff[b]:aoff[b + 1]], re)
        cd.append(r["cd"])
        ld.append(r["ld"])
        sep.append(r["sep"].reshape(-1))
    return np.concatenate(cd), np.concatenate(ld), np.concatenate(sep)


@pytest.mark.parametrize("formulation", [0, 1], ids=["stream", "hess_smith"])
def test_thwaites_matches_oracle_on_the_gpu_surface_speed(formulation):
    _say(f"viscous correction, formulation {formulation}")
    w = synth.random_workload(61, 48, n_choices=(64, 128, 200, 256, 300, 400, 512), k_max=3)
    re = 3e6
    xy, gamma, cl, bl = _run(w, formulation, re)
    cd, ld, sep = _oracle_layer(w, xy, gamma, cl, re)
    e_cd = np.max(np.abs(bl["cd"] - cd) / np.abs(cd))
    e_ld = np.max(np.abs(bl["ld"] - ld) / np.maximum(1.0, np.abs(ld)))
    _say(f"  cd {np.min(cd):.2e}..{np.max(cd):.2e}, rel err cd {e_cd:.1e}, ld {e_ld:.1e}, "
         f"separations attached {np.mean(sep == -1):.2f}")
    assert e_cd < 1e-12 and e_ld < 1e-12
    assert np.array_equal(bl["sep"], sep)


def test_thwaites_end_to_end_against_the_oracle():
    # oracle solve + oracle layer on the same nodes: within the solve's bound
    _say("viscous correction end to end, ga2048[:64]")
    w = synth.workload("ga2048", B=64)
    re = 1e6
    xy, gamma, cl, bl = _run(w, 0, re)
    ref = oracle.solve_batch(xy, w.node_offsets(), w.alpha_flat(), w.alpha_offsets())
    cd, ld, sep = _oracle_layer(w, xy, ref["gamma"], ref["cl"], re)
    e = np.max(np.abs(bl["cd"] - cd) / np.abs(cd))
    _say(f"  rel err cd {e:.1e}")
    assert e < 1e-9
    assert np.array_equal(bl["sep"], sep)


def test_thwaites_cylinder_closed_form_on_the_gpu():
    # Hess-Smith surface speed on a 512-gon (exact at the midpoints): the
    # drag converges to Thwaites' closed form for the cylinder,
    # Cd sqrt(Re_D) = 5.64365 (quadrature of the closed-form shear up to
    # separation at 103.11 degrees; pinned in the oracle's tests)
    import torch
    import paper_1511_02166_amd as P
    _say("viscous correction, cylinder")
    N, re = 512, 2e5
    xy_flat, noff = synth.pack_nodes([synth.circle_nodes(N, R=0.5)])
    s = P.PanelSolver(noff, np.array([0, 1], dtype=np.int32), 0, formulation=P.PANEL_HESS_SMITH)
    s.solve(torch.as_tensor(xy_flat, device="cuda"), torch.zeros(1, dtype=torch.float64, device="cuda"))
    bl = s.viscous(re)
    torch.cuda.synchronize()
    cdre = float(bl["cd"][0]) * math.sqrt(re)
    _say(f"  Cd sqrt(Re) = {cdre:.6f}, separation panels {bl['sep'].cpu().numpy()}")
    assert abs(cdre / 5.643645758556941 - 1) < 1e-4
    ju, jl = (int(x) for x in bl["sep"].cpu().numpy())
    assert ju + jl == N - 1
    phi = 180.0 - 360.0 * (ju + 0.5) / N
    assert abs(phi - 103.11) < 1.5 * 360.0 / N
