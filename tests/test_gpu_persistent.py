"""The persistent step kernel (ppmb_batch_step modes 3 and 4): every brick's
three passes and the step's dt in one launch of resident waves that take
items in order and wait on per-brick counters.  It must give the per-stage
launches' states, dts and counters bit for bit: with both pass orders,
with the dt taken from the previous step's fused maxima and after a state
change (CFL reduction first), when the fused maximum falls below its band
(the redo reduction inside the kernel), on sphere bricks with solid cells
skipped, and replayed from a HIP graph."""
import math

import numpy as np
import pytest

from paper_1810_13416_amd import problems as pr

pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="the persistent step kernel is switched off: its launches did not "
                                      "complete on the GPU (test timed out in synchronize) and the cause "
                                      "is not found; ppmb_batch_step modes 3 and 4 return INVALID")]


def make_batch(probs, prec, states=None):
    from paper_1810_13416_amd import ppmb
    B = ppmb.Batch([p.params for p in probs], ppmb.FP64 if prec == "fp64" else ppmb.FP32)
    for b, p in enumerate(probs):
        B.set_state(b, p.state if states is None else states[b])
    return B


def snapshot(B, nb):
    B.synchronize()
    return ([B.get_conserved(b) for b in range(nb)], [B.last_dt(b) for b in range(nb)], B.counters()[:3])


def assert_same(a, b, nb):
    (sa, da, ca), (sb, db, cb) = a, b
    assert da == db
    assert ca == cb
    for k in range(nb):
        for q in range(15):
            assert np.array_equal(sa[k][q], sb[k][q]), (k, q)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_persistent_step_equals_per_stage_launches(prec):
    probs = pr.bricks(count=12, seed=41, nmin=8, nmax=24)
    nb = len(probs)
    ref = make_batch(probs, prec)
    ref.step(0.8, 5, mode=0)
    want = snapshot(ref, nb)
    for mode in (3, 4):
        B = make_batch(probs, prec)
        B.step(0.8, 5, mode=mode)
        assert_same(snapshot(B, nb), want, nb)
        B.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_persistent_step_with_sphere_bricks_and_a_falling_maximum(prec):
    # a sphere brick (solid cells skipped after the first pass), a ball
    # brick with one fast cell whose speed spreads out (the fused maximum
    # drops below its band: the redo reduction runs inside the kernel) and
    # two plain bricks
    ball = pr.ball(24)
    st = [a.copy() for a in ball.state]
    st[1][12, 12, 12] = 0.8 * math.sqrt(5.0 / 3.0 * 0.7 / 1.3)
    probs = [pr.config3(n=24), ball] + pr.bricks(count=2, seed=3, nmin=8, nmax=16)
    states = [probs[0].state, st, probs[2].state, probs[3].state]
    nb = len(probs)
    ref = make_batch(probs, prec, states)
    ref.step(0.8, 4, mode=0)
    want = snapshot(ref, nb)
    for mode in (3, 4):
        B = make_batch(probs, prec, states)
        B.step(0.8, 4, mode=mode)
        assert_same(snapshot(B, nb), want, nb)
        B.close()


def test_persistent_graph_replays_with_eager_work_between():
    # the captured persistent steps replayed several times, with eager
    # persistent and per-stage steps and a state change in between
    probs = pr.bricks(count=6, seed=5, nmin=8, nmax=20)
    nb = len(probs)
    A = make_batch(probs, "fp32")
    G = make_batch(probs, "fp32")
    for k, mode in ((2, 4), (3, 3), (2, 4), (1, 0), (4, 4)):
        A.step(0.8, k, mode=0)
        G.step(0.8, k, mode=mode)
        assert_same(snapshot(G, nb), snapshot(A, nb), nb)
    fresh = pr.bricks(count=6, seed=6, nmin=8, nmax=20)
    for b in range(nb):
        if fresh[b].params.n == probs[b].params.n:
            A.set_state(b, fresh[b].state)
            G.set_state(b, fresh[b].state)
    A.step(0.8, 4, mode=0)
    G.step(0.8, 4, mode=4)
    assert_same(snapshot(G, nb), snapshot(A, nb), nb)


def test_persistent_step_falls_back_where_it_does_not_apply():
    # with shock dissipation the step takes the per-stage launches: same bits
    probs = pr.bricks(count=4, seed=8, nmin=8, nmax=16)
    nb = len(probs)
    A = make_batch(probs, "fp32")
    B = make_batch(probs, "fp32")
    A.set_shock_dissipation(0.1)
    B.set_shock_dissipation(0.1)
    A.step(0.8, 3, mode=0)
    B.step(0.8, 3, mode=3)
    assert_same(snapshot(B, nb), snapshot(A, nb), nb)
