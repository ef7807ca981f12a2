"""Parity at the full benchmark size: the spherical shell at 512^3, in the
launch configuration bench.py times (default pass shapes, FP32 perturbation
form, and the FP64 form).  The oracle cannot step 134 M cells in a test, but
a 1-D pass changes a cell only through its own pencil, so one pass of the
GPU over the whole grid is checked on sampled pencils, each recomputed by
the oracle as a one-pencil grid with the same coordinates, boundaries,
gravity, base state and sphere, from the GPU's own input values for that
pencil.  The time step at full size is checked by a property that holds at
any size: the dt that the last pass's fused reduction gives equals the CFL
kernel's dt on the same state, bit for bit.

Tolerances: FP64 as every FP64 parity test (relative L1 1e-12, Linf 1e-9
of the field's scale over the sampled pencils; measured 3e-16).  FP32
against the FP64 oracle from identical FP32-representable inputs, one
pass: relative L1 and Linf 1e-5, the FP32 figure for smooth flows (measured
1.5e-7 and 3.7e-7: the FP32 arithmetic and one rounding of each stored
value, no branch of the constraints resolved differently).  The flattening
depends only on the pencil too, so FP64 passes with it on are checked the
same way on the shell with a planted shock at its centre."""
import numpy as np
import pytest

import oracle
from paper_1810_13416_amd import problems as pr

pytestmark = pytest.mark.gpu

N = 512
# (a, b): the two transverse indices of a pencil, in axis order; through
# the centre, off-centre, near the sphere's surface, fully solid, next to
# a cube face, and at random places
SAMPLES = [(255, 255), (256, 250), (300, 128), (255, 20), (0, 0), (511, 256), (100, 400), (417, 63)]


def _pencil_params(params, axis, a, b):
    dx = params.dx
    t = [ax for ax in range(3) if ax != axis]
    n = [1, 1, 1]
    n[axis] = params.n[axis]
    org = list(params.origin)
    for ax, idx in zip(t, (a, b)):
        org[ax] = params.origin[ax] + idx * dx
    P = pr.GridParams(**{**params.__dict__})
    P.n = tuple(n)
    P.origin = tuple(org)
    return P


def _pencils(S, axis):
    """FP64 copies of the 15 conserved fields of every sampled pencil."""
    off, fs, plane, px = S.layout()
    raw = S.current_state_tensor()
    stride = (1, px, plane)[axis]
    out = []
    for a, b in SAMPLES:
        base = {0: a * px + b * plane, 1: a + b * plane, 2: a + b * px}[axis]
        fields = []
        for q in range(15):
            s0 = off + q * fs + base
            fields.append(raw[s0: s0 + (N - 1) * stride + 1: stride].double().cpu().numpy())
        out.append(fields)
    return out


def _shape(axis):
    return {0: (1, 1, N), 1: (1, N, 1), 2: (N, 1, 1)}[axis]


def _scales(ref):
    """Per field: (L1 scale, max scale) over all sampled pencils; the fv
    moments share f0's scale, the momenta their common scale."""
    out = []
    for q in range(15):
        group = [5] if q >= 5 else ([1, 2, 3] if q in (1, 2, 3) else [q])
        l1 = sum(float(np.sum(np.abs(p[g]))) for p in ref for g in group) / len(group)
        li = max(float(np.max(np.abs(p[g]))) for p in ref for g in group)
        out.append((max(l1, 1e-300), max(li, 1e-300)))
    return out


def _check_pass(S, prob, axis, l1_tol, li_tol, flat=False):
    dt = S.dt(prob.cfl)
    before = _pencils(S, axis)
    S.pass_(axis, dt)
    after = _pencils(S, axis)
    ref = []
    flagged = 0
    for (a, b), cons in zip(SAMPLES, before):
        O = oracle.Oracle(_pencil_params(prob.params, axis, a, b), threads=1)
        O.set_conserved([c.reshape(_shape(axis)) for c in cons])
        if flat:
            # the coefficients depend on the pencil alone
            O.set_flattening(True)
            flagged += int(np.count_nonzero(O.flattening(axis)))
        O.pass_(axis, dt)
        ref.append([c.reshape(-1) for c in O.get_conserved()])
        O.close()
    # the pass did change the sampled fluid cells (the check is not vacuous)
    moved = max(float(np.max(np.abs(o[q] - c[q]))) for o, c in zip(ref, before) for q in (0, 4))
    assert moved > 0.0
    sc = _scales(ref)
    worst = (0.0, 0.0)
    for q in range(15):
        e1 = sum(float(np.sum(np.abs(g[q] - o[q]))) for g, o in zip(after, ref)) / sc[q][0]
        ei = max(float(np.max(np.abs(g[q] - o[q]))) for g, o in zip(after, ref)) / sc[q][1]
        assert e1 <= l1_tol and ei <= li_tol, (axis, q, e1, ei)
        worst = (max(worst[0], e1), max(worst[1], ei))
    if flat:
        assert flagged > 0                 # the flattening acted on the samples
    print(f"axis {axis}: worst relative L1 {worst[0]:.3e}, Linf {worst[1]:.3e}")


@pytest.fixture(scope="module")
def shell():
    return pr.config3(n=N)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_fullsize_passes_match_oracle_on_sampled_pencils(shell, prec):
    from paper_1810_13416_amd import ppmb
    S = ppmb.Sim(shell.params, ppmb.FP32 if prec == "fp32" else ppmb.FP64)
    S.set_state(shell.state)
    tol = (1e-5, 1e-5) if prec == "fp32" else (1e-12, 1e-9)
    # the first pass after set_state writes every cell, the later ones skip
    # the solid cells beyond the stencil reach: the x pass runs both ways
    for axis in (0, 1, 2, 0):
        _check_pass(S, shell, axis, *tol)
    S.close()


def test_fullsize_flattened_passes_match_oracle_on_sampled_pencils_fp64(shell):
    # the shell with a planted shock: the central pressure doubled inside
    # r < 0.06 and a converging flow -0.5 x inside r < 0.3, so that the
    # pencils through the centre have flattened cells
    from paper_1810_13416_amd import ppmb
    P = shell.params
    z, y, x = np.meshgrid(*(pr._centres(P, ax) for ax in (2, 1, 0)), indexing="ij")
    r2 = (x * x + y * y) + z * z
    _, p0c = oracle.base_profile(P, np.array([0.0]))
    st = list(shell.state)
    st[4] = st[4] + np.where(r2 < 0.06 ** 2, float(p0c[0]), 0.0)
    inner = r2 < 0.3 ** 2
    for d, c in ((1, x), (2, y), (3, z)):
        st[d] = st[d] + np.where(inner, -0.5 * c, 0.0)
    del x, y, z, r2, inner
    S = ppmb.Sim(P, ppmb.FP64)
    S.set_state(st)
    del st
    S.set_flattening(True)
    for axis in (0, 1, 2):
        _check_pass(S, shell, axis, 1e-12, 1e-9, flat=True)
    S.close()


def test_fullsize_fused_dt_equals_cfl_kernel(shell):
    from paper_1810_13416_amd import ppmb
    A = ppmb.Sim(shell.params, ppmb.FP32)
    A.set_state(shell.state)
    A.step_auto(shell.cfl, 2)
    cons = A.get_conserved()
    nstep = A.nstep
    A.step_auto(shell.cfl, 1)            # dt from the maxima the previous step's last pass folded in
    fused = A.last_dt()
    A.close()
    B = ppmb.Sim(shell.params, ppmb.FP32)
    B.set_conserved(cons)
    B.nstep = nstep
    del cons
    assert B.dt(shell.cfl) == fused
    B.close()


def test_fullsize_brick_batch_matches_oracle_on_sampled_bricks():
    # the 256-brick workload of the benchmark (FP32, autotuned launch shape,
    # graph replay): one step, sampled bricks against the oracle from the
    # same FP32-representable inputs and the GPU's per-brick dt; density
    # and energy compared as full fields (base added back), as the FP32
    # figure is defined
    from paper_1810_13416_amd import ppmb
    probs = pr.bricks()
    B = ppmb.Batch([p.params for p in probs], ppmb.FP32)
    for b, p in enumerate(probs):
        B.set_state(b, p.state)
    B.autotune(0.8, reps=1)
    picks = [0, 17, 101, 200, 255]
    start = {b: B.get_conserved(b) for b in picks}
    B.step(0.8, 1, mode=1)
    B.synchronize()
    for b in picks:
        O = oracle.Oracle(probs[b].params, threads=8)
        O.set_conserved(start[b])
        O.step(B.last_dt(b))
        ref = O.get_conserved()
        got = B.get_conserved(b)
        r0, p0 = O.base()
        gm1 = probs[b].params.gamma - 1.0
        for c in (ref, got):
            c[0] = c[0] + r0
            c[4] = c[4] + p0 / gm1
        O.close()
        for q in range(15):
            group = [5] if q >= 5 else ([1, 2, 3] if q in (1, 2, 3) else [q])
            l1 = max(sum(float(np.sum(np.abs(ref[g]))) for g in group) / len(group), 1e-300)
            li = max(max(float(np.max(np.abs(ref[g]))) for g in group), 1e-300)
            d = np.abs(got[q] - ref[q])
            assert float(np.sum(d)) / l1 <= 1e-5 and float(np.max(d)) / li <= 1e-5, (b, q)
    B.close()
