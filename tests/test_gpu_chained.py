"""Chained (not reseeded) FP64 runs of flow into the confining sphere's wall
against the oracle: eight steps, plain, with the shock dissipation and with
the flattening, each side stepping from its own state with the oracle's dt.
The per-step tests (test_gpu_shock, test_gpu_flatten) reseed the GPU from
the oracle every step, since a limiter or Riemann-branch decision can flip
on a last-bit difference between the two evaluation orders and move a cell
by far more than rounding; chained, no decision flips on this flow, and the
whole run meets the FP64 bar (relative L1 <= 1e-12 per field group, Linf <=
1e-9 of the group's largest value); the count of cells beyond 1e-9 is
printed beside it."""
import numpy as np
import pytest

import oracle
from paper_1810_13416_amd import problems as pr

pytestmark = pytest.mark.gpu


def wall_ball(n=20):
    prob = pr.ball(n)
    prob.state[1][:] = 0.3
    prob.state[2][:] = -0.2
    prob.state[3][:] = 0.1
    return prob


@pytest.mark.parametrize("mode", ["plain", "dissipation", "flattening"])
def test_chained_wall_flow_matches_oracle(mode):
    from paper_1810_13416_amd import ppmb
    prob = wall_ball()
    S = ppmb.Sim(prob.params, ppmb.FP64)
    S.set_state(prob.state)
    O = oracle.Oracle(prob.params, threads=8)
    O.set_conserved(S.get_conserved())
    if mode != "plain":
        S.set_shock_dissipation(0.1)
        O.set_dissipation(0.1)
    if mode == "flattening":
        S.set_flattening(True)
        O.set_flattening(True)
    for _ in range(8):
        dt = O.dt(prob.cfl)
        O.step(dt)
        S.step(dt)
    a, b = S.get_conserved(), O.get_conserved()
    report = []
    for q in range(15):
        g = [5] if q >= 5 else ([1, 2, 3] if q in (1, 2, 3) else [q])
        s1 = max(sum(float(np.sum(np.abs(b[x]))) for x in g) / len(g), 1e-300)
        si = max(max(float(np.max(np.abs(b[x]))) for x in g), 1e-300)
        d = np.abs(a[q] - b[q])
        report.append((q, float(np.sum(d)) / s1, float(np.max(d)) / si, int(np.count_nonzero(d > 1e-9 * si))))
    print(f"{mode}: (field, relL1, relLinf, cells beyond 1e-9) of {a[0].size}:", report)
    for q, l1, li, far in report:
        assert l1 <= 1e-12 and li <= 1e-9, (q, l1, li, far)
