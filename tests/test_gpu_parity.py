"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs.  Tolerances: FP64 relative L1 <= 1e-12 and relative
Linf <= 1e-9 per field (contraction and evaluation order only change
rounding); FP32 perturbation form against the FP64 oracle relative L1 <= 1e-5
and relative Linf <= 1e-4 on smooth flows."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_1810_13416_amd import problems as pr

pytestmark = pytest.mark.gpu

ODD_X = {1, 6, 12, 14}


def sim(params, prec="fp64"):
    from paper_1810_13416_amd import ppmb
    return ppmb.Sim(params, ppmb.FP64 if prec == "fp64" else ppmb.FP32)


def orc(params):
    return oracle.Oracle(params, threads=8)


def rel_l1(a, b):
    den = np.sum(np.abs(b))
    return float(np.sum(np.abs(a - b)) / den) if den > 0 else float(np.sum(np.abs(a - b)))


def rel_linf(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a - b)))


def scale_of(oa, q):
    """Natural scale of field q: the fv moments share the scale of f0, the
    three momentum components the scale of the momentum vector."""
    if q >= 5:
        ref = [oa[5]]
    elif q in (1, 2, 3):
        ref = [oa[1], oa[2], oa[3]]
    else:
        ref = [oa[q]]
    l1 = sum(float(np.sum(np.abs(r))) for r in ref) / len(ref)
    li = max(float(np.max(np.abs(r))) for r in ref)
    return max(l1, 1e-300), max(li, 1e-300)


def compare(ga, oa, l1, linf, fields=range(15), label=""):
    worst = []
    for q in fields:
        s1, si = scale_of(oa, q)
        d = np.abs(ga[q] - oa[q])
        e1, ei = float(np.sum(d)) / s1, float(np.max(d)) / si
        worst.append((q, e1, ei))
        assert e1 <= l1 and ei <= linf, (label, q, e1, ei)
    return worst


def full_fields(state, base):
    """rho, p (full) and the rest unchanged, for FP32-vs-FP64 comparisons."""
    r0, p0 = base
    out = list(state)
    out[0] = state[0] + r0
    out[4] = state[4] + p0
    return out


def test_library_loads_on_gpu():
    from paper_1810_13416_amd import ppmb
    import torch
    assert torch.cuda.is_available()
    ppmb.load()


# the x pass has two kernels (lanes along x, or the marching kernel with
# lanes across y); the y and z passes have only the marching kernel
@pytest.mark.parametrize("axis,xshape", [(0, "lanes"), (0, "march"), (1, "lanes"), (2, "lanes")])
@pytest.mark.parametrize("shape", [(20, 24, 28), (67, 5, 9), (130, 3, 4), (5, 13, 7)])
def test_single_pass_matches_oracle(axis, shape, xshape, monkeypatch):
    if xshape == "march":
        monkeypatch.setenv("PPMB_X_MARCH", "1")
    # one pass on a ragged grid (not a multiple of the 64-lane tile)
    P = pr.config1(n=8).params
    P = dataclasses.replace(P, n=shape, dx=1.0 / max(shape))
    rng = np.random.default_rng(3)
    st = []
    for q in range(15):
        if q == 0:
            st.append(1.0 + 0.1 * rng.standard_normal(P.shape))
        elif q == 4:
            st.append(1.0 + 0.1 * rng.standard_normal(P.shape))
        elif q in (1, 2, 3):
            st.append(0.2 * rng.standard_normal(P.shape))
        elif q == 5:
            st.append(rng.uniform(0.0, 1.0, P.shape))
        else:
            st.append(0.02 * rng.standard_normal(P.shape))
    O = orc(P)
    O.set_state(st)
    S = sim(P)
    S.set_state(st)
    dt = 0.5 * O.dt(0.8)
    O.pass_(axis, dt)
    S.pass_(axis, dt)
    compare(S.get_conserved(), O.get_conserved(), 1e-13, 1e-11, label=f"pass {axis}")


def test_config1_fp64_20_steps_matches_oracle():
    prob = pr.config1()
    O = orc(prob.params)
    O.set_state(prob.state)
    S = sim(prob.params)
    S.set_state(prob.state)
    # the same state gives the same dt to 2 ulp
    dto, dtg = O.dt(prob.cfl), S.dt(prob.cfl)
    assert abs(dtg - dto) <= 2 * np.spacing(dto)
    for _ in range(prob.nsteps):
        dto = O.dt(prob.cfl)
        O.step(dto)
        S.step(dto)
    compare(S.get_state(), O.get_state(), 1e-12, 1e-9, label="config1")
    tg, to = S.totals(), O.totals()
    assert np.allclose(tg, to, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("cfg", ["strat", "sphere"])
def test_stratified_fp64_matches_oracle(cfg):
    prob = pr.config2(n=24) if cfg == "strat" else pr.config3(n=32)
    O = orc(prob.params)
    O.set_state(prob.state)
    S = sim(prob.params)
    S.set_state(prob.state)
    rb, pb = O.base()
    gr, gp = S.base()
    assert rel_linf(gr, rb) <= 1e-14 and rel_linf(gp, pb) <= 1e-14
    for _ in range(6):
        dt = O.dt(prob.cfl)
        O.step(dt)
        S.step(dt)
    go, oo = full_fields(S.get_state(), (gr, gp)), full_fields(O.get_state(), (rb, pb))
    compare(go, oo, 1e-12, 1e-9, label=cfg)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("base", ["none", "const"])
def test_uniform_state_bitwise(prec, base):
    prob = pr.uniform(base=base)
    S = sim(prob.params, prec)
    S.set_state(prob.state)
    before = S.get_conserved()
    S.run(10, 0.8)
    after = S.get_conserved()
    for q in range(6):
        assert np.array_equal(before[q], after[q]), q


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("cfg", ["strat", "sphere"])
def test_hydrostatic_exact_on_gpu(prec, cfg):
    prob = pr.config2(n=24) if cfg == "strat" else pr.config3(n=24)
    prob.params.heat_kind = 0
    st = [np.zeros_like(a) for a in prob.state[:5]] + prob.state[5:]
    S = sim(prob.params, prec)
    S.set_state(st)
    S.run(20, 0.8)
    c = S.get_conserved()
    for q in range(5):
        assert np.all(c[q] == 0.0), q


def test_fp32_perturbation_matches_fp64_oracle_on_smooth_flow():
    # the smooth-flow precision target: 100 steps, relative L1 <= 1e-5
    prob = pr.config1(base="const")
    O = orc(prob.params)
    O.set_state(prob.state)
    S = sim(prob.params, "fp32")
    S.set_state(prob.state)
    for _ in range(100):
        dt = O.dt(prob.cfl)
        O.step(dt)
        S.step(dt)
    ones = (np.ones(prob.params.shape), np.ones(prob.params.shape))
    ga, oa = S.get_state(), O.get_state()
    worst = compare(full_fields(ga, ones), full_fields(oa, ones), 1e-5, 1e-4,
                    fields=range(6), label="fp32 smooth")
    print("fp32 vs fp64 oracle, 100 steps (field, relL1, relLinf):", worst)
    # the stored perturbations themselves (rho', p' of order 1e-2 here):
    # errors relative to the perturbation, the quantity the form keeps
    pert = {q: (rel_l1(ga[q], oa[q]), rel_linf(ga[q], oa[q])) for q in (0, 4)}
    print("perturbation-relative (rho', p'):", pert)
    for q, (e1, ei) in pert.items():
        assert e1 <= 1e-4 and ei <= 1e-3, (q, e1, ei)


def test_conservation_on_gpu():
    for prec, tol in (("fp64", 1e-13), ("fp32", 1e-6)):
        prob = pr.config1(base="const" if prec == "fp32" else "none")
        S = sim(prob.params, prec)
        S.set_state(prob.state)
        t0 = S.totals()
        S.step_auto(prob.cfl, 20)
        t1 = S.totals()
        assert abs(t1[0] - t0[0]) <= tol * t0[0], prec
        assert abs(t1[4] - t0[4]) <= tol * t0[4], prec


def test_mirror_symmetry_fp64():
    prob = pr.config1()

    def mirror(st):
        return [(-1.0 if q in ODD_X else 1.0) * np.ascontiguousarray(a[:, :, ::-1]) for q, a in enumerate(st)]
    sym = [0.5 * (a + b) for a, b in zip(prob.state, mirror(prob.state))]
    S = sim(prob.params)
    S.set_state(sym)
    S.run(20, 0.8)
    c = S.get_conserved()
    compare(mirror(c), c, 1e-12, 1e-10, fields=range(6), label="mirror")


def test_step_auto_equals_host_dt_loop_and_is_deterministic():
    prob = pr.config2(n=16)
    A = sim(prob.params, "fp32")
    A.set_state(prob.state)
    A.step_auto(prob.cfl, 5)
    B = sim(prob.params, "fp32")
    B.set_state(prob.state)
    B.run(5, prob.cfl)
    C = sim(prob.params, "fp32")
    C.set_state(prob.state)
    C.step_auto(prob.cfl, 5)
    for a, b, c in zip(A.get_conserved(), B.get_conserved(), C.get_conserved()):
        assert np.array_equal(a, b) and np.array_equal(a, c)
    assert np.array_equal(A.totals(), C.totals())


def test_checkpoint_resume_bitwise_on_gpu():
    prob = pr.config2(n=16)
    A = sim(prob.params)
    A.set_state(prob.state)
    A.step_auto(prob.cfl, 6)
    B = sim(prob.params)
    B.set_state(prob.state)
    B.step_auto(prob.cfl, 3)
    ck, k = B.get_conserved(), B.nstep
    C = sim(prob.params)
    C.set_conserved(ck)
    C.nstep = k
    C.step_auto(prob.cfl, 3)
    for a, c in zip(A.get_conserved(), C.get_conserved()):
        assert np.array_equal(a, c)


def test_sod_fp64_matches_oracle():
    prob = pr.sod(200)
    O = orc(prob.params)
    O.set_state(prob.state)
    S = sim(prob.params)
    S.set_state(prob.state)
    for _ in range(40):
        dt = O.dt(0.8)
        O.step(dt)
        S.step(dt)
    compare(S.get_state(), O.get_state(), 1e-12, 1e-9, fields=(0, 1, 4, 5), label="sod")


def test_nonphysical_state_is_reported():
    from paper_1810_13416_amd import ppmb
    prob = pr.uniform()
    st = [a.copy() for a in prob.state]
    st[4][3, 2, 1] = -1.0      # negative pressure in one cell
    S = sim(prob.params)
    S.set_state(st)
    with pytest.raises(ppmb.PPMBError, match="-4"):
        S.dt(0.8)


def test_counters_match_oracle_fp64():
    prob = pr.config1(n=24)
    O = orc(prob.params)
    O.set_state(prob.state)
    S = sim(prob.params)
    S.set_state(prob.state)
    for _ in range(5):
        dt = O.dt(0.8)
        O.step(dt)
        S.step(dt)
    co, cg = O.counters(), S.counters()
    assert cg[3] == co[3] == 5
    assert cg[0] == co[0] and cg[2] == co[2]
    assert abs(cg[1] - co[1]) <= 1e-4 * co[1]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_fused_cfl_reduction_equals_cfl_kernel(prec):
    # the last pass of a step folds the next step's CFL maxima in; the dt
    # it gives must be the CFL kernel's dt on the same state, bit for bit
    # (sphere: solid cells excluded; heating in the last pass)
    prob = pr.config3(n=24)
    A = sim(prob.params, prec)
    A.set_state(prob.state)
    A.step_auto(prob.cfl, 3)
    B = sim(prob.params, prec)
    B.set_state(prob.state)
    B.step_auto(prob.cfl, 2)
    assert A.last_dt() == B.dt(prob.cfl)
    # after a state change the next step recomputes from the state
    C = sim(prob.params, prec)
    C.set_state(prob.state)
    C.step_auto(prob.cfl, 1)
    C.set_state(prob.state)
    C.step_auto(prob.cfl, 1)
    D = sim(prob.params, prec)
    D.set_state(prob.state)
    assert C.last_dt() == D.dt(prob.cfl)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_fused_cfl_reduction_falls_back_when_the_maximum_drops(prec):
    # one fast cell in a gas at rest: after a step its speed has spread out
    # and the maximum falls far below the band under the previous maximum
    # inside which the last pass evaluates speeds exactly; the next dt must
    # still be the CFL kernel's, bit for bit
    prob = pr.ball(24)
    st = [a.copy() for a in prob.state]
    c0 = math.sqrt(5.0 / 3.0 * 0.7 / 1.3)
    st[1][12, 12, 12] = 0.8 * c0
    A = sim(prob.params, prec)
    A.set_state(st)
    d0 = A.dt(prob.cfl)
    A.step_auto(prob.cfl, 1)
    d1 = A.dt(prob.cfl)
    assert d1 > d0 * 1.05               # the maximum did drop by more than the band
    B = sim(prob.params, prec)
    B.set_state(st)
    B.step_auto(prob.cfl, 3)
    C = sim(prob.params, prec)
    C.set_state(st)
    C.step_auto(prob.cfl, 2)
    assert B.last_dt() == C.dt(prob.cfl)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_device_state_layout_is_the_documented_pitched_one(prec):
    # rows padded to 64 elements, padded field stride: reading the raw device
    # buffer through ppmb_state_layout gives the conserved fields
    prob = pr.config1(n=20)
    S = sim(prob.params, prec)
    S.set_state(prob.state)
    S.step_auto(prob.cfl, 1)
    off, fs, plane, px = S.layout()
    nz, ny, nx = S.shape
    assert px % 64 == 0 and px >= nx and plane == px * ny and fs >= nz * plane
    raw = S.current_state_tensor().cpu().numpy()
    cons = S.get_conserved()
    for q in range(15):
        a = raw[off + q * fs: off + q * fs + nz * plane].reshape(nz, ny, px)[:, :, :nx]
        assert np.array_equal(a.astype(np.float64), cons[q]), q


def test_fp32_strong_shock_riemann_resolve_matches_oracle():
    # Sec. 1 (32-bit sweeps on perturbations): a Riemann problem whose FP32
    # iteration has not converged in two steps is solved again in FP64.  A
    # pressure jump of 10 (FP32-representable data) forces that fallback;
    # every field after one pass per axis is compared with the FP64 oracle
    prob = pr.blast(24, p_in=10.0)
    for axis in range(3):
        O = orc(prob.params)
        O.set_state(prob.state)
        S = sim(prob.params, "fp32")
        S.set_state(prob.state)
        dt = O.dt(0.8)
        O.pass_(axis, dt)
        S.pass_(axis, dt)
        c = S.counters()
        assert c[2] > 0, c                 # the FP64 re-solve ran
        assert O.counters()[2] == 0        # FP64 Newton converged everywhere
        worst = compare(S.get_state(), O.get_state(), 1e-5, 1e-4, label=f"fp32 blast axis {axis}")
        print(f"axis {axis}: {c[2]} FP64 re-solves; (field, relL1, relLinf):", worst[:6])


def test_fp32_stratified_box_matches_fp64_oracle():
    # the case the perturbation form exists for (Sec. 1): a stratified base
    # (density falling 10x over the box), Mach 0.03 flow, heating, light
    # fluid on top; 100 steps in FP32 against the FP64 oracle
    prob = pr.config2(n=32, noise=0.0)
    O = orc(prob.params)
    O.set_state(prob.state)
    S = sim(prob.params, "fp32")
    S.set_state(prob.state)
    for _ in range(100):
        dt = O.dt(prob.cfl)
        O.step(dt)
        S.step(dt)
    base = O.base()
    ga, oa = S.get_state(), O.get_state()
    worst = compare(full_fields(ga, base), full_fields(oa, base), 1e-5, 1e-4, label="fp32 stratified")
    pert = {q: (rel_l1(ga[q], oa[q]), rel_linf(ga[q], oa[q])) for q in (0, 4)}
    print("fp32 stratified vs oracle (field, relL1, relLinf):", worst[:6])
    print("perturbation-relative (rho', p'):", pert)
    for q, (e1, ei) in pert.items():
        assert e1 <= 1e-3 and ei <= 1e-2, (q, e1, ei)
