"""Throughput of the PPM + PPB 3-D step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-fp64] [--no-cpu]
                    [--no-bricks] [--no-accuracy] [--no-ppb2d] [--calib-copy-mib M]

Workload: the spherical convection shell on a 512^3 grid (FP32 perturbation
form on an FP64 radial hydrostatic base, radial gravity, heating, confining
sphere, seeded velocity noise), one step = three 1-D PPM+PPB passes plus the
FP64 CFL reduction and heating, with dt computed on the device.  Inputs are
resident in HBM before timing starts.  Prints ONE JSON line.

The JSON carries
  roofline      the dominant kernel (the pass kernel with the largest time
                per step) against the HBM peak: algorithmic bytes per launch
                (15 fields read + 15 written per cell) over its average
                duration, timed with HIP events on the library's stream
                inside the timed region; `traffic` is the measured HBM bytes
                per launch from the committed hardware-counter summary, or
                null when the pass sources differ from the ones counted;
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same recipe;
  fp64          the same grid and steps in FP64 on the same GPU;
  bricks        256 independent bricks (16..64 cells per axis) advanced
                together in FP32: one launch per stage for all bricks, the
                same replayed from a HIP graph, and one launch per stage and
                brick, after the launch-shape autotuner; the same bricks in
                FP64, and the FP32 batch against the FP64 one after the same
                fixed-dt steps;
  accuracy      the stratified box at 128^3 in FP32 and FP64 against the
                same at 256^3 in FP64 (fixed dt, restricted to 128^3): the
                FP32 round-off error against the truncation error;
  ppb2d         the slotted-disk advection test of Fig. 3 (2-D PPB, FP32,
                100^2 cells, 1 / 10 / 100 revolutions: shape error, mass,
                bounds) and the throughput of its pass kernel on 4096^2.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "sweep_traffic_shell512_fp32.txt")
SQ_SUMMARY = os.path.join(ROOT, "profiles", "sweep_sq_counters_shell512_fp32.md")
# VALU issue peak without packed FP32 (disabled in every HIP unit here): 256 CUs x 4
# SIMDs x 16 lanes per cycle x 2.4 GHz, in 10^12 lane-instructions per second
VALU_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12
FP32_PEAK_TFLOPS = 157.3                       # MI355X vector FP32, published (packed instructions)
FP32_NONPACKED_TFLOPS = 2 * VALU_PEAK_T        # one FMA per lane per cycle without them
# the kernels behind each pass of the FP32 step
PASS_KERNELS = {"x": "sweep_x_kernel<float, false, false>", "y": "sweep_kernel<float, 1, false, false>",
                "z": "sweep_kernel<float, 2, false, false>"}
N_FIELDS = 15
# algorithmic bytes per updated cell and pass (FP32): the 15 state fields read
# and written once, and the base rho0 and p0 (working precision) read once
BYTES_PER_CELL_PASS = (2 * N_FIELDS + 2) * 4
METRIC = "cell-updates/s per PPM+PPB 3-D step, FP32-perturb vs FP64, % HBM roofline"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_rotation(sim, n, reps=5):
    """The spin-up increment and the spherical-shell sums on the bench state:
    time per call (HIP events on the library's stream) and algorithmic HBM
    rate over the fluid cells, the only ones either touches.  FP32 state:
    the increment reads rho', m_x, m_y, E' and the FP64 rho0 and writes m_x,
    m_y, E' (36 B per fluid cell); the shell sums read rho', m (3), f0 and
    rho0 (28 B per fluid cell)."""
    import torch
    st = sim.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(reps):
        sim.spin_add(1e-3)
    e1.record(st)
    torch.cuda.synchronize()
    spin_ms = e0.elapsed_time(e1) / reps
    nbins, dr = n // 2, 2.0 / n               # shells of width dx out to the sphere r = 1
    first = sim.shell_profile(nbins, dr)      # workspace allocation outside the timing
    cells = int(round(first[:, 0].sum() / dr ** 3))
    torch.cuda.synchronize()
    e0.record(st)
    prof = sim.shell_profile(nbins, dr)
    e1.record(st)
    torch.cuda.synchronize()
    shell_ms = e0.elapsed_time(e1)
    vol = float(prof[:, 0].sum())
    return {"fluid_cells": cells,
            "spin_add": {"ms": spin_ms, "bytes_per_cell": 36,
                         "achieved_GBs": 36 * cells / (spin_ms * 1e-3) / 1e9},
            "shell_profile": {"ms": shell_ms, "bins": nbins, "bytes_per_cell": 28,
                              "achieved_GBs": 28 * cells / (shell_ms * 1e-3) / 1e9,
                              "fluid_volume_over_4pi_3": vol / (4.0 * math.pi / 3.0)}}


TILING = (256, 2)      # cells per wave along a pencil (0: whole), x rows per wave


def run_gpu(prob, precision, steps, warmup, dev_prims, rotation=False, dissk=0.0, flat=False, skip=True):
    import torch
    from paper_1810_13416_amd import ppmb
    sim = ppmb.Sim(prob.params, precision, device="cuda:0")
    sim.set_solid_skip(skip)
    sim.set_tiling(*TILING)
    sim.set_state_device(dev_prims)
    if dissk > 0.0:
        sim.set_shock_dissipation(dissk)
    if flat:
        sim.set_flattening(True)
    torch.cuda.synchronize()
    sim.step_auto(prob.cfl, warmup)
    torch.cuda.synchronize()
    sim.profile(True)
    # the timed steps in up to 5 blocks of equal length, each bracketed by
    # events on the library's stream; ms per step is the median block's
    nblk = max(1, min(5, steps))
    sizes = [steps // nblk + (1 if b < steps % nblk else 0) for b in range(nblk)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nblk + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(sim.stream)
    for b, k in enumerate(sizes):
        sim.step_auto(prob.cfl, k)
        ev[b + 1].record(sim.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.profile(False)
    counts, ms = sim.profile_read()
    per_block = [ev[b].elapsed_time(ev[b + 1]) / k for b, k in enumerate(sizes)]
    ms_step = float(sorted(per_block)[len(per_block) // 2]) if nblk % 2 else \
        0.5 * sum(sorted(per_block)[nblk // 2 - 1: nblk // 2 + 1])
    tot = sim.totals()
    cnt = sim.counters()
    info = {"ms_per_step": ms_step, "ms_per_step_blocks": per_block,
            "ms_per_step_mean": ev[0].elapsed_time(ev[-1]) / steps, "wall_ms_per_step": 1e3 * wall / steps,
            "pass_ms": {ax: (ms[i] / counts[i] if counts[i] else None) for i, ax in enumerate("xyz")},
            "totals": [float(v) for v in tot], "counters": cnt, "dt_last": sim.last_dt()}
    if rotation:
        info["rotation"] = run_rotation(sim, prob.params.n[0])
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return info


CONFIG5_SUMMARY = os.path.join(ROOT, "profiles", "config5_shell1024_fp32_vs_fp64.json")


def run_config5(n=1024, steps=20, warmup=3, slab=64):
    """The spherical shell at 1024^3 (the 512^3 recipe at half the cell
    width) in FP32 and then in FP64 on the same GPU.  Both are filled plane
    slab by plane slab (the FP64 primitives of the whole grid would take
    129 GB of host memory) and advanced by the same warmup + steps steps of
    one fixed dt (the FP32 state's dt at Courant number 0.6), timed; the
    FP32 state is then kept on the host in FP32 and compared field by field
    with the FP64 state: relative L1 = sum |a - b| / sum |b| and
    relative Linf = max |a - b| / max |b| with rho and p as full fields
    (base added back), velocities against the largest speed component and
    the fv moments against f0's scale; the perturbation-relative L1 of rho'
    and p' besides.  After the comparison each precision is timed for
    `steps` more steps with dt computed on the device (the bench's step)."""
    import numpy as np
    import torch
    from paper_1810_13416_amd import ppmb, problems
    P = problems.config3_params(n)
    out = {"grid": [n] * 3, "cells": n ** 3, "steps": steps, "warmup": warmup, "tiling": list(TILING)}
    kept, base, dt = None, None, None
    slabs = [(k0, min(slab, n - k0)) for k0 in range(0, n, slab)]
    for prec, name in ((ppmb.FP32, "fp32"), (ppmb.FP64, "fp64")):
        t0 = time.perf_counter()
        try:
            S = ppmb.Sim(P, prec, device="cuda:0")
        except (ppmb.PPMBError, RuntimeError) as e:     # the grid does not fit
            out[name] = {"error": str(e)[:300]}
            log(f"config5 {name}: {e}")
            torch.cuda.empty_cache()
            continue
        S.set_tiling(*TILING)
        for k0, nk in slabs:
            S.set_state_planes(k0, problems.config3_planes(n, k0, nk))
            log(f"config5 {name}: planes {k0}..{k0 + nk - 1} set")
        log(f"config5 {name}: state set in {time.perf_counter() - t0:.0f} s")
        if dt is None:
            dt = S.dt(0.6)
            out["dt_fixed"] = dt
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(warmup):
            S.step(dt)
        torch.cuda.synchronize()
        e0.record(S.stream)
        for _ in range(steps):
            S.step(dt)
        e1.record(S.stream)
        torch.cuda.synchronize()
        ms_fixed = e0.elapsed_time(e1) / steps
        tot = [float(v) for v in S.totals()]
        log(f"config5 {name}: {ms_fixed:.2f} ms/step at fixed dt")
        if name == "fp32":
            kept = [[a.astype(np.float32) for a in S.get_state_planes(k0, nk)] for k0, nk in slabs]
            base = S.base()
        elif kept is not None:
            r0, p0 = base
            acc = np.zeros((15, 4))          # sum |d|, sum |b|, max |d|, max |b| (full fields)
            pert = np.zeros((2, 2))          # rho', p': sum |d|, sum |b|
            for s_i, (k0, nk) in enumerate(slabs):
                b = S.get_state_planes(k0, nk)
                a = [x.astype(np.float64) for x in kept[s_i]]
                kept[s_i] = None
                for i, q in enumerate((0, 4)):
                    pert[i] += (np.abs(a[q] - b[q]).sum(), np.abs(b[q]).sum())
                a[0] += r0[k0:k0 + nk]
                b[0] += r0[k0:k0 + nk]
                a[4] += p0[k0:k0 + nk]
                b[4] += p0[k0:k0 + nk]
                for q in range(15):
                    d = np.abs(a[q] - b[q])
                    acc[q] += (d.sum(), np.abs(b[q]).sum(), 0.0, 0.0)
                    acc[q, 2] = max(acc[q, 2], float(d.max()))
                    acc[q, 3] = max(acc[q, 3], float(np.abs(b[q]).max()))
            err = {}
            for q in range(15):
                grp = [5] if q >= 5 else ([1, 2, 3] if q in (1, 2, 3) else [q])
                l1 = sum(acc[g, 1] for g in grp) / len(grp)
                li = max(acc[g, 3] for g in grp)
                err[problems.FIELD_NAMES[q]] = {"relL1": acc[q, 0] / max(l1, 1e-300),
                                                "relLinf": acc[q, 2] / max(li, 1e-300)}
            out["fp32_vs_fp64"] = err
            out["perturbation_relL1"] = {"rho'": pert[0, 0] / max(pert[0, 1], 1e-300),
                                         "p'": pert[1, 0] / max(pert[1, 1], 1e-300)}
            log("config5: compared")
        S.step_auto(0.8, 1)
        torch.cuda.synchronize()
        e0.record(S.stream)
        S.step_auto(0.8, steps)
        e1.record(S.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[name] = {"ms_per_step": ms, "cell_updates_per_s": n ** 3 / (ms * 1e-3),
                     "ms_per_step_fixed_dt": ms_fixed, "dt_last": S.last_dt(), "totals_after_fixed_dt": tot}
        log(f"config5 {name}: {ms:.2f} ms/step with device dt")
        S.close()
        del S
        torch.cuda.empty_cache()
    if "fp32" in out and "fp64" in out and "ms_per_step" in out["fp64"] and "ms_per_step" in out["fp32"]:
        out["speedup_fp32_over_fp64"] = out["fp64"]["ms_per_step"] / out["fp32"]["ms_per_step"]
    return out


def measured_traffic():
    """Measured HBM bytes per launch of each pass kernel, from the committed
    counter summary, if it was taken from the pass sources as they are now."""
    from paper_1810_13416_amd import profsum
    try:
        info = profsum.read_traffic_summary(TRAFFIC_SUMMARY)
    except OSError:
        return None
    if info.get("sweep_sources_sha256") != profsum.sweep_sources_hash():
        return None
    return info


def measured_valu():
    """VALU instructions per launch of each pass kernel, from the committed
    SQ counter summary, if it was taken from the pass sources as they are now."""
    from paper_1810_13416_amd import profsum
    try:
        info = profsum.read_counters_summary(SQ_SUMMARY)
    except OSError:
        return None
    if info.get("sweep_sources_sha256") != profsum.sweep_sources_hash():
        return None
    return info


def calib_copy(mib):
    """One plain elementwise copy kernel (read M MiB, write M MiB): the
    reference dispatch against which hardware byte counters are scaled."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.neg(a, out=b)
    torch.cuda.synchronize()
    log(f"calibration copy: {n * 4} bytes read, {n * 4} bytes written")
    del a, b
    torch.cuda.empty_cache()


def run_bricks(steps, warmup, fp64=True):
    """The batched-brick workload in each launch mode (FP32), and with
    `fp64` the same in FP64 against it."""
    import numpy as np
    import torch
    from paper_1810_13416_amd import ppmb, problems
    probs = problems.bricks()
    cells = int(sum(int(np.prod(p.params.n)) for p in probs))
    cfl = 0.8
    out = {"bricks": len(probs), "cells": cells, "modes": {}}
    shape = None
    for mode, name in ((0, "batched"), (1, "graph"), (2, "per_brick")):
        B = ppmb.Batch([p.params for p in probs], ppmb.FP32)
        for b, p in enumerate(probs):
            B.set_state(b, p.state)
        if shape is None:
            shape = B.autotune(cfl, reps=2)
            tiling = B.tiling()
            out["autotuned_shape"] = {"march_waves": shape[0], "x_waves": shape[1],
                                      "march_chunk": tiling[0], "x_rows": tiling[1]}
        else:
            B.set_shape(*shape)
            B.set_tiling(*tiling)
        B.step(cfl, warmup, mode)
        B.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(B.stream)
        B.step(cfl, steps, mode)
        e1.record(B.stream)
        B.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out["modes"][name] = {"ms_per_step": ms, "cell_updates_per_s": cells / (ms * 1e-3)}
        log(f"bricks {name}: {ms:.3f} ms/step")
        B.close()
        del B
        torch.cuda.empty_cache()
    if fp64:
        out["fp64"] = run_bricks_fp64(probs, cells, steps, warmup, cfl, shape, tiling)
        out["fp64"]["speedup_fp32_batched_over_fp64"] = \
            out["fp64"]["ms_per_step"] / out["modes"]["batched"]["ms_per_step"]
    return out


def run_bricks_fp64(probs, cells, steps, warmup, cfl, shape, tiling, nfixed=10):
    """The bricks in FP64: the batched step's time, and the FP32 batch
    against the FP64 one after the same `nfixed` steps of one fixed dt (half
    the smallest brick dt at Courant 0.8 of the FP64 initial state): per
    field the relative L1 difference of the conserved fields (the fv
    moments against f0's scale, momenta against the momentum vector's),
    the largest over the bricks."""
    import numpy as np
    import torch
    from paper_1810_13416_amd import ppmb
    nb = len(probs)

    def batch(prec):
        B = ppmb.Batch([p.params for p in probs], prec)
        for b, p in enumerate(probs):
            B.set_state(b, p.state)
        B.set_shape(*shape)
        B.set_tiling(*tiling)
        return B
    B = batch(ppmb.FP64)
    B.step(cfl, warmup, 0)
    B.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(B.stream)
    B.step(cfl, steps, 0)
    e1.record(B.stream)
    B.synchronize()
    ms = e0.elapsed_time(e1) / steps
    log(f"bricks fp64 batched: {ms:.3f} ms/step")
    B.close()
    del B
    # equal accuracy: both precisions over the same fixed-dt steps
    T = batch(ppmb.FP64)
    T.step(cfl, 1, 0)
    dt = 0.5 * min(T.last_dt(b) for b in range(nb))
    T.close()
    del T
    # fresh batches: both start at step 0 (the pass order alternates with
    # the step number)
    R = batch(ppmb.FP64)
    A = batch(ppmb.FP32)
    for _ in range(nfixed):
        A.step_dt(dt)
        R.step_dt(dt)
    A.synchronize()
    R.synchronize()
    kinds = sorted(set(p.name for p in probs))
    worst = {k: np.zeros(15) for k in kinds}
    for b in range(nb):
        a, r = A.get_conserved(b), R.get_conserved(b)
        w = worst[probs[b].name]
        for q in range(15):
            grp = [5] if q >= 5 else ([1, 2, 3] if q in (1, 2, 3) else [q])
            s1 = sum(float(np.sum(np.abs(r[x]))) for x in grp) / len(grp)
            w[q] = max(w[q], float(np.sum(np.abs(a[q] - r[q]))) / max(s1, 1e-300))
    A.close()
    R.close()
    del A, R
    torch.cuda.empty_cache()
    names = ["rho'", "m_x", "m_y", "m_z", "E'", "f0", "fx", "fy", "fz", "fxx", "fyy", "fzz", "fxy", "fyz", "fzx"]
    for k in kinds:
        log(f"bricks {k} fp32 vs fp64 after {nfixed} steps: worst relative L1 {max(worst[k]):.2e}")
    return {"ms_per_step": ms, "cell_updates_per_s": cells / (ms * 1e-3), "fixed_dt": dt, "fixed_steps": nfixed,
            "fp32_vs_fp64_relL1_worst_brick": {k: {names[q]: float(worst[k][q]) for q in range(15)} for k in kinds},
            "note": "brick_sine: periodic sine flows (rho' and E' start at zero, so their scale is the small "
                    "compressive part of the flow); brick_strat: stratified boxes with seeded per-cell noise"}


def _restrict(a):
    """Average 2x2x2 blocks (z, y, x arrays)."""
    n0, n1, n2 = a.shape
    return a.reshape(n0 // 2, 2, n1 // 2, 2, n2 // 2, 2).mean(axis=(1, 3, 5))


def run_accuracy(nsteps=200):
    """FP32 round-off against truncation error on the stratified box."""
    import numpy as np
    from paper_1810_13416_amd import ppmb, problems
    # no per-cell noise: both resolutions sample the same continuous flow
    fine = problems.config2(n=256, noise=0.0)
    coarse = problems.config2(n=128, noise=0.0)
    F = ppmb.Sim(fine.params, ppmb.FP64, device="cuda:0")
    F.set_state(fine.state)
    dt = F.dt(fine.cfl)                 # CFL 0.8 on the fine grid, used by all runs
    for _ in range(nsteps):
        F.step(dt)
    sf = F.get_state()
    bf0, _ = F.base()
    F.close()
    del F, fine
    res = {}
    for prec, name in ((ppmb.FP64, "fp64"), (ppmb.FP32, "fp32")):
        C = ppmb.Sim(coarse.params, prec, device="cuda:0")
        C.set_state(coarse.state)
        for _ in range(nsteps):
            C.step(dt)
        res[name] = C.get_state()
        if name == "fp64":
            bc0, _ = C.base()
        C.close()
        del C

    def rel(a, b):
        return float(np.sum(np.abs(a - b)) / max(np.sum(np.abs(b)), 1e-300))

    fields = {"u_x": 1, "u_y": 2, "u_z": 3, "p'": 4}
    out = {"grid": "128^3 vs 256^3 restricted", "steps": nsteps, "dt": dt, "fields": {}}
    worst = 0.0
    for k, q in fields.items():
        trunc = rel(res["fp64"][q], _restrict(sf[q]))
        rnd = rel(res["fp32"][q], res["fp64"][q])
        out["fields"][k] = {"truncation_relL1": trunc, "fp32_roundoff_relL1": rnd,
                            "ratio": rnd / trunc if trunc > 0 else None}
        if trunc > 0:
            worst = max(worst, rnd / trunc)
    rho_c = bc0 + res["fp64"][0]
    rho_f = bf0 + sf[0]
    out["fields"]["rho"] = {"truncation_relL1": rel(rho_c, _restrict(rho_f)),
                            "fp32_roundoff_relL1": rel(bc0 + res["fp32"][0], rho_c)}
    out["worst_velocity_pressure_ratio"] = worst
    out["equal_accuracy"] = bool(worst <= 0.1)
    return out


def run_ppb2d():
    """The slotted-disk test and the 2-D PPB pass kernel's throughput."""
    import numpy as np
    import torch
    from paper_1810_13416_amd import ppmb, problems
    z = problems.zalesak(100)
    nrev = int(round(1.0 / z.dt(0.5)))
    dt = 1.0 / nrev
    G = ppmb.PPB2D(z.n, z.dx, z.origin, z.centre, z.omega, ppmb.FP32)
    G.set(z.coef)
    g0 = z.coef[0]
    out = {"grid": [100, 100], "steps_per_revolution": nrev, "precision": "fp32", "revolutions": {}}
    done = 0
    for rev in (1, 10, 100):
        G.steps(dt, (rev - done) * nrev)
        done = rev
        f = G.get()[0]
        out["revolutions"][str(rev)] = {"shape_L1_over_area": float(np.abs(f - g0).sum() / g0.sum()),
                                         "mass_drift": float(f.sum() / g0.sum() - 1.0),
                                         "fv_min": float(f.min()), "fv_max": float(f.max())}
        log(f"ppb2d: {rev} revolution(s), shape error {out['revolutions'][str(rev)]['shape_L1_over_area']:.4f}")
    G.close()
    # throughput of the pass kernel on a large grid
    n = 4096
    coef = problems.slotted_disk_moments(n, depth=4)
    G = ppmb.PPB2D((n, n), 1.0 / n, (0.0, 0.0), (0.5, 0.5), 2.0 * np.pi, ppmb.FP32)
    G.set(coef)
    del coef
    dtb = 0.5 * (1.0 / n) / (2.0 * np.pi * 0.5)
    G.steps(dtb, 3)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    steps = 50
    e0.record(G.stream)
    G.steps(dtb, steps)
    e1.record(G.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    G.close()
    cells = n * n
    gbs = 2 * (2 * 6 * 4 * cells) / (ms * 1e-3) / 1e9      # two passes per step
    out["throughput"] = {"grid": [n, n], "ms_per_step": ms, "cell_updates_per_s": cells / (ms * 1e-3),
                         "bytes_per_cell_per_pass": 48, "achieved_GBs": gbs, "frac_hbm": gbs / HBM_PEAK_GBS}
    log(f"ppb2d {n}^2: {ms:.3f} ms/step, {gbs:.0f} GB/s")
    return out


def _oracle_rate(n, steps, threads):
    import oracle
    from paper_1810_13416_amd import problems
    prob = problems.config3(n=n)
    O = oracle.Oracle(prob.params, threads=threads)
    O.set_state(prob.state)
    del prob.state
    t0 = time.perf_counter()
    for _ in range(steps):
        O.step(O.dt(0.8))
    dt = time.perf_counter() - t0
    O.close()
    return n ** 3 * steps / dt, dt


def cpu_baseline(n=512, steps=2, n1=128, steps1=2):
    """The FP64 oracle on the host cores: the benchmark's own grid for a
    few steps with every core, and a smaller grid of the same recipe on
    one thread."""
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    rate, dt = _oracle_rate(n, steps, threads)
    log(f"oracle {n}^3 x {steps} on {threads} threads: {dt:.1f} s")
    rate1, dt1 = _oracle_rate(n1, steps1, 1)
    log(f"oracle {n1}^3 x {steps1} on 1 thread: {dt1:.1f} s")
    return {"value": rate, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle, the same shell at {n}^3, {steps} step(s), {dt:.1f} s on {threads} threads",
            "seconds": dt,
            "single_thread": {"value": rate1, "unit": "cell-updates/s", "cores": 1,
                              "sample": f"FP64 oracle, the same recipe at {n1}^3, {steps1} step(s), {dt1:.1f} s"}}


def fluid_cell_count(params):
    """Cells whose centre lies inside the confining sphere, by the library's
    test: (x^2 + y^2) + z^2 below the square of the radius (radius 1 here,
    whose square and correctly rounded square root are exact)."""
    import numpy as np
    if not params.sphere:
        return int(np.prod(params.n))
    assert params.sphere_r == 1.0
    c = [params.origin[a] + (np.arange(params.n[a]) + 0.5) * params.dx for a in range(3)]
    xy = (c[0][None, :] * c[0][None, :]) + (c[1][:, None] * c[1][:, None])
    return int(sum(int(np.count_nonzero(xy + z * z < 1.0)) for z in c[2]))


def main():
    global TILING
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-bricks", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-ppb2d", action="store_true")
    ap.add_argument("--no-rotation", action="store_true")
    ap.add_argument("--tiling", type=str, default=None,
                    help="march_chunk,x_rows of the pass kernels (default: %s,%s)" % TILING)
    ap.add_argument("--config5", action="store_true",
                    help="run the 1024^3 FP32-vs-FP64 comparison and write its summary (JSON)")
    ap.add_argument("--config5-out", default=CONFIG5_SUMMARY,
                    help="where --config5 writes its summary (default: the committed one in profiles/)")
    ap.add_argument("--compare-skip", action="store_true",
                    help="also time the FP32 step with every pass writing every cell")
    ap.add_argument("--bricks-only", action="store_true",
                    help="time only the batched-brick workload and print its summary (for profiling its kernels)")
    ap.add_argument("--calib-copy-mib", type=int, default=0)
    ap.add_argument("--dissipation", type=float, default=0.1,
                    help="coefficient of the extra FP32 runs with shock handling (0: skip them)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU brick decomposition is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1810_13416_amd import ppmb, problems

    if args.tiling:
        TILING = tuple(int(v) for v in args.tiling.split(","))
    if args.calib_copy_mib:
        calib_copy(args.calib_copy_mib)
    if args.config5:
        res = run_config5()
        res["command"] = "python bench.py --config5"
        res["sweep_sources_sha256"] = __import__("paper_1810_13416_amd.profsum", fromlist=["x"]).sweep_sources_hash()
        with open(args.config5_out, "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps(res), flush=True)
        return
    if args.bricks_only:
        res = run_bricks(args.steps, args.warmup, fp64=not args.no_fp64)
        print(json.dumps(res), flush=True)
        return
    log(f"generating the {args.n}^3 shell inputs")
    t0 = time.perf_counter()
    prob = problems.config3(n=args.n)
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s; uploading")
    dev = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0") for a in prob.state]
    prob.state = None
    torch.cuda.synchronize()
    cells = args.n ** 3

    log("FP32 run")
    r32 = run_gpu(prob, ppmb.FP32, args.steps, args.warmup, dev, rotation=not args.no_rotation)
    log(f"FP32: {r32['ms_per_step']:.3f} ms/step, passes {r32['pass_ms']}")
    rall = None
    if args.compare_skip:
        log("FP32 run, every pass writing every cell")
        rall = run_gpu(prob, ppmb.FP32, args.steps, args.warmup, dev, skip=False)
        log(f"FP32 all cells: {rall['ms_per_step']:.3f} ms/step, passes {rall['pass_ms']}")
    rdiss = rflat = None
    if args.dissipation > 0.0:
        log(f"FP32 run with shock dissipation K = {args.dissipation}")
        rdiss = run_gpu(prob, ppmb.FP32, max(5, args.steps // 2), args.warmup, dev, dissk=args.dissipation)
        log(f"FP32 dissipative: {rdiss['ms_per_step']:.3f} ms/step, passes {rdiss['pass_ms']}")
        log("FP32 run with shock dissipation and flattening")
        rflat = run_gpu(prob, ppmb.FP32, max(5, args.steps // 2), args.warmup, dev, dissk=args.dissipation,
                        flat=True)
        log(f"FP32 dissipation + flattening: {rflat['ms_per_step']:.3f} ms/step, passes {rflat['pass_ms']}")
    r64 = None
    if not args.no_fp64:
        log("FP64 run")
        r64 = run_gpu(prob, ppmb.FP64, max(2, args.steps // 4), 1, dev)
        log(f"FP64: {r64['ms_per_step']:.3f} ms/step")
    del dev
    torch.cuda.empty_cache()

    value = cells / (r32["ms_per_step"] * 1e-3)
    fluid = fluid_cell_count(prob.params)
    # algorithmic bytes of a pass: the 15 fields read and written once and
    # the two base fields read once for every cell it updates, the fluid
    # cells (solid cells keep their values and are not moved); ghost reads
    # and the solid cells near the fluid that a pass does touch are
    # traffic, not algorithmic bytes
    bytes_per_launch = BYTES_PER_CELL_PASS * fluid
    kernels = {}
    for ax, ms in r32["pass_ms"].items():
        if ms:
            kernels[PASS_KERNELS[ax]] = {"avg_launch_ms": ms,
                                         "achieved_GBs": bytes_per_launch / (ms * 1e-3) / 1e9}
    dom_ax = max((ax for ax in r32["pass_ms"] if r32["pass_ms"][ax]), key=lambda a: r32["pass_ms"][a])
    dom = PASS_KERNELS[dom_ax]
    achieved = kernels[dom]["achieved_GBs"]
    tr = measured_traffic()
    traffic = None
    if tr and dom in tr.get("bytes_per_launch", {}):
        traffic = tr["bytes_per_launch"][dom]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"spherical convection shell {args.n}^3, FP32 perturbation on FP64 "
                               "radial base, radial gravity, heating r<0.2, confining sphere, "
                               "velocity noise 1e-4 c0; step = 3 passes + FP64 CFL dt on device",
                   "cells": cells, "grid": [args.n] * 3, "precision": "fp32-perturbation"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": dom, "bytes_per_launch": bytes_per_launch,
                     "avg_launch_ms": kernels[dom]["avg_launch_ms"], "kernels": kernels,
                     "traffic_source": os.path.relpath(TRAFFIC_SUMMARY, ROOT) if traffic else None},
        "hbm_roofline_cell_updates_per_s": HBM_PEAK_GBS * 1e9 / (3 * BYTES_PER_CELL_PASS),
        "fraction_of_hbm_roofline": value / (HBM_PEAK_GBS * 1e9 / (3 * BYTES_PER_CELL_PASS)),
        "fluid": {"cells": fluid, "cell_updates_per_s": fluid / (r32["ms_per_step"] * 1e-3),
                  "fraction_of_hbm_roofline": fluid / (r32["ms_per_step"] * 1e-3) /
                  (HBM_PEAK_GBS * 1e9 / (3 * BYTES_PER_CELL_PASS)),
                  "note": "the cells the method updates; value counts every cell of the grid, "
                          "solid cells (kept, and skipped by the passes beyond the stencil reach) included"},
        "ms_per_step_blocks": r32["ms_per_step_blocks"], "ms_per_step_mean": r32["ms_per_step_mean"],
        "counters": r32["counters"],
    }
    valu = measured_valu()
    if valu:
        # VALU issue (lane-instructions) and VALU FLOPs (an FMA counts 2, a
        # transcendental 1) per launch, from the committed counter summary,
        # over the live launch duration; per fluid cell, the cells updated
        per, flop = {}, {}
        for k, v in kernels.items():
            cs = valu["kernels"].get(k, {})
            n = cs.get("SQ_INSTS_VALU")
            t = v["avg_launch_ms"] * 1e-3
            if n:
                per[k] = {"valu_per_fluid_cell": 64 * n / fluid, "achieved": 64 * n / t / 1e12}
            f = 0.0
            for prec in ("F32", "F64"):
                f += sum(cs.get(f"SQ_INSTS_VALU_{op}_{prec}", 0.0) for op in ("ADD", "MUL", "TRANS"))
                f += 2.0 * cs.get(f"SQ_INSTS_VALU_FMA_{prec}", 0.0)
            if f:
                flop[k] = {"flop_per_fluid_cell": 64 * f / fluid, "achieved_TFLOPs": 64 * f / t / 1e12}
        if dom in per:
            out["roofline_alu"] = {"bound": "alu", "kernel": dom, "achieved": per[dom]["achieved"],
                                   "peak": VALU_PEAK_T, "unit": "T VALU lane-instructions/s",
                                   "frac": per[dom]["achieved"] / VALU_PEAK_T, "kernels": per,
                                   "source": os.path.relpath(SQ_SUMMARY, ROOT)}
        if dom in flop:
            out["roofline_valu_flops"] = {
                "bound": "alu", "kernel": dom, "achieved": flop[dom]["achieved_TFLOPs"], "unit": "TFLOP/s",
                "peak": FP32_PEAK_TFLOPS, "frac": flop[dom]["achieved_TFLOPs"] / FP32_PEAK_TFLOPS,
                "peak_nonpacked": FP32_NONPACKED_TFLOPS,
                "frac_nonpacked": flop[dom]["achieved_TFLOPs"] / FP32_NONPACKED_TFLOPS,
                "kernels": flop, "source": os.path.relpath(SQ_SUMMARY, ROOT)}
    if "rotation" in r32:
        out["rotation"] = r32["rotation"]
        log(f"spin-up increment {r32['rotation']['spin_add']['ms']:.3f} ms, shell sums "
            f"{r32['rotation']['shell_profile']['ms']:.3f} ms")
    if rall:
        out["without_solid_skip"] = {"ms_per_step": rall["ms_per_step"], "pass_ms": rall["pass_ms"],
                                     "speedup_of_skip": rall["ms_per_step"] / r32["ms_per_step"]}
    if rdiss:
        out["shock_dissipation"] = {"k": args.dissipation, "value": cells / (rdiss["ms_per_step"] * 1e-3),
                                    "unit": "cell-updates/s", "ms_per_step": rdiss["ms_per_step"],
                                    "pass_ms": rdiss["pass_ms"],
                                    "slowdown_vs_plain": rdiss["ms_per_step"] / r32["ms_per_step"]}
    if rflat:
        out["shock_dissipation_and_flattening"] = {
            "k": args.dissipation, "value": cells / (rflat["ms_per_step"] * 1e-3), "unit": "cell-updates/s",
            "ms_per_step": rflat["ms_per_step"], "pass_ms": rflat["pass_ms"],
            "slowdown_vs_plain": rflat["ms_per_step"] / r32["ms_per_step"]}
    if r64:
        out["fp64"] = {"value": cells / (r64["ms_per_step"] * 1e-3), "unit": "cell-updates/s",
                       "ms_per_step": r64["ms_per_step"], "pass_ms": r64["pass_ms"],
                       "speedup_fp32_over_fp64": r64["ms_per_step"] / r32["ms_per_step"]}
    if not args.no_bricks:
        log("batched bricks")
        out["bricks"] = run_bricks(max(5, args.steps // 2), 2, fp64=not args.no_fp64)
    if not args.no_accuracy:
        log("accuracy: FP32 round-off vs truncation error")
        out["accuracy"] = run_accuracy()
    if not args.no_ppb2d:
        log("2-D PPB: slotted disk")
        out["ppb2d"] = run_ppb2d()
    if os.path.exists(CONFIG5_SUMMARY):
        with open(CONFIG5_SUMMARY) as f:
            c5 = json.load(f)
        c5["source"] = os.path.relpath(CONFIG5_SUMMARY, ROOT)
        c5["taken_from_current_sources"] = c5.get("sweep_sources_sha256") == \
            __import__("paper_1810_13416_amd.profsum", fromlist=["x"]).sweep_sources_hash()
        out["config5_1024"] = c5
    if not args.no_cpu:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
