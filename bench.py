"""Benchmark of the D2Q9 lattice Boltzmann hot path on one MI355X.

Default workload: one-fluid flow through a seeded porous medium of
4096 x 4096 nodes (non-overlapping discs, radius 8..24, porosity 0.6,
periodic, tau = 0.8, acceleration 1e-5 along e1), FP32 shifted storage.
A step is one time step (stream + bounce-back + collide) over the whole
lattice; the step kernel fuses five of them per launch (the first four kept
in LDS), so each launch advances five steps.

Prints ONE JSON line with MLUPS (all nodes), the HBM roofline of the step
kernel (algorithmic bytes of the steps one launch advances / measured launch
time, beside the bytes the launch must move at least), the FP64 CPU
oracle timed on a bounded sample of the same workload, and variants:
16-bit storage, the two-component Shan-Chen + solute + growth step, and the
batched ensemble of uneven lattices against running them one at a time.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D2Q9 MLUPS + % of HBM roofline; FP16-store & batched vs plain FP32"
PEAK_HBM_GBPS = 8000.0
STORE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash():
    """Hash of the code the one-fluid step kernel is built from: the shared
    parameter header and the device code up to the general step."""
    csrc = os.path.join(ROOT, "paper_1202_0442_amd", "csrc")
    h = hashlib.sha256()
    with open(os.path.join(csrc, "lb2d_common.hpp"), "rb") as fh:
        hdr = fh.read()
    h.update(hdr[hdr.index(b"struct PlainLattice"):hdr.index(b"struct FullParams")])
    with open(os.path.join(csrc, "lb2d_device.hpp"), "rb") as fh:
        src = fh.read()
    h.update(src[:src.index(b"// --------------------------------------------------------- general step")])
    return h.hexdigest()[:16]


def measured_traffic(name):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel and workload, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)\s+source:\s*([0-9a-f]+)", txt)
    if not m or m.group(2) != source_hash():
        return None
    return float(m.group(1))


def make_porous_lattice(lb2d, w, storage, stream, rounding="nearest", accel=None):
    L = lb2d.Lattice(0)
    L.lattice("d2q9", w.nx, w.ny, w.tau)
    if rounding != "nearest":
        L.rounding(rounding, 2012)
    L.boundary_style("noslip")
    for (xc, yc, r) in w.discs:
        L.obstacle_circle(xc, yc, r)
    for r in w.rects:
        L.obstacle_rect(*r)
    L.aveacceleration(1, w.accel_x if accel is None else accel)
    L.bind(storage, stream=stream)
    return L


# warm-up steps before a timed region: two 60-step graphs, so that graph
# capture and instantiation happen outside it
GRAPH_WARMUP = 120


def time_steps(torch, stream, fn, steps):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fn(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def _oracle_rate(n, threads, target_seconds):
    """MLUPS of the FP64 oracle, as it stands, on an n x n sample of the
    porous workload (same generator, seed and parameters)."""
    from oracle import Oracle
    from oracle.oracle import set_threads
    from paper_1202_0442_amd import inputs
    used = set_threads(threads)
    w = inputs.porous(n=n, seed=2)
    o = Oracle(w.nx, w.ny)
    o.fluids(1, w.tau)
    for (xc, yc, r) in w.discs:
        o.obstacle_circle(xc, yc, r)
    o.aveacceleration(1, w.accel_x)
    o.set_fields(0, 1.0)
    o.iteration(2)
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < target_seconds:
        o.iteration(5)
        steps += 5
    dt = time.perf_counter() - t0
    sample = (f"porous {w.nx}x{w.ny} (discs r 8..24, porosity 0.6, seed 2), {steps} steps, {dt:.1f} s, "
              f"FP64 plain C, {used} thread{'s' if used > 1 else ''}")
    return w.nx * w.ny * steps / dt / 1e6, used, sample


def _oracle_timed(o, nodes, target_seconds):
    """MLUPS of an oracle lattice over about target_seconds (after 2 steps)."""
    o.iteration(2)
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < target_seconds:
        o.iteration(5)
        steps += 5
    dt = time.perf_counter() - t0
    return nodes * steps / dt / 1e6, steps, dt


def _oracle_configs(target_seconds):
    """The FP64 oracle on one thread on the other configurations (or samples
    of them): the 128x64 FP64 channel, the two-component + solute + reaction
    workload on a 256x256 sample of its generator, and one lattice of the
    ensemble."""
    import numpy as np
    from oracle import Oracle
    from oracle.oracle import set_threads
    from paper_1202_0442_amd import inputs
    set_threads(1)
    out = {}
    w = inputs.poiseuille()
    o = Oracle(w.nx, w.ny)
    o.fluids(1, w.tau)
    for r in w.rects:
        o.obstacle_rect(*r)
    o.aveacceleration(1, w.accel_x)
    o.set_fields(0, 1.0)
    v, n, dt = _oracle_timed(o, w.nx * w.ny, target_seconds)
    out["channel"] = {"value": v, "unit": "MLUPS", "sample": f"channel {w.nx}x{w.ny} (the full configuration), "
                                                             f"{n} steps, {dt:.1f} s, 1 thread"}
    w = inputs.sc_solute(n=256)
    e = w.extra
    ra, rb = inputs.sc_initial_fields(w)
    o = Oracle(w.nx, w.ny)
    o.fluids(2, w.tau, e["tau2"])
    o.interforce(e["G"])
    o.adhesiveforce(e["Gads"][0], 0)
    o.adhesiveforce(e["Gads"][1], 1)
    for d in w.discs:
        o.obstacle_circle(*d)
    o.set_fields(0, ra.ravel())
    o.set_fields(1, rb.ravel())
    o.solute(e["tau_s"], 9)
    o.solute_opening("xlo", "dirichlet", e["C_in"])
    o.solute_opening("xhi", "adiabatic", 0.0)
    o.surface_reaction(e["kr"], e["Cs"], e["b0"], e["bmax"], e["rng_seed"])
    o.set_concentration(np.zeros(w.nx * w.ny))
    v, n, dt = _oracle_timed(o, w.nx * w.ny, target_seconds)
    out["sc_solute"] = {"value": v, "unit": "MLUPS",
                        "sample": f"two-component + D2Q9 solute + reaction, {w.nx}x{w.ny} sample of the 2048x2048 "
                                  f"generator, {n} steps, {dt:.1f} s, 1 thread"}
    w = next(x for x in inputs.ensemble() if max(x.nx, x.ny) <= 512)
    o = Oracle(w.nx, w.ny)
    o.fluids(1, w.tau)
    for d in w.discs:
        o.obstacle_circle(*d)
    o.aveacceleration(1, w.accel_x)
    o.set_fields(0, 1.0)
    v, n, dt = _oracle_timed(o, w.nx * w.ny, target_seconds)
    out["ensemble_lattice"] = {"value": v, "unit": "MLUPS",
                               "sample": f"one ensemble lattice, {w.nx}x{w.ny}, {n} steps, {dt:.1f} s, 1 thread"}
    return out


def cpu_baseline(target_seconds=15.0):
    """The FP64 oracle on one host thread (the reported baseline), the same
    oracle with its OpenMP rows over the host threads this process may use
    on a larger sample, and the oracle on one thread on the other
    configurations."""
    v1, _, s1 = _oracle_rate(512, 1, target_seconds)
    nthr = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    vn, used, sn = _oracle_rate(1024, nthr, 8.0)
    return {"value": v1, "unit": "MLUPS", "cores": 1, "kind": "oracle", "sample": s1,
            "all_threads": {"value": vn, "unit": "MLUPS", "cores": used, "sample": sn},
            "per_configuration": _oracle_configs(4.0)}


def steady_k(L, accel, tau, chunk=1000, rel=1e-6, max_steps=100000):
    """Steps the lattice until its permeability k = nu <u_x>_all / a_x
    changes by less than rel over `chunk` steps; (k, steps, converged)."""
    nu = (tau - 0.5) / 3.0
    prev = None
    while L.step_count() < max_steps:
        L.iteration(chunk)
        _, ux, _ = L.moments(0)
        k = nu * float(ux.mean()) / accel
        if prev is not None and abs(k - prev) <= rel * abs(k):
            return k, L.step_count(), True
        prev = k
    return None, L.step_count(), False


def permeability(lb2d, w, L, stream):
    """Permeability of the porous workload from runs driven to steady state
    (after the timed steps): at the workload's forcing, on the benchmark's
    lattice, and at twice it on a fresh lattice of the same geometry (Darcy's
    law: the same k).  k is null when a run does not settle."""
    k1, n1, ok1 = steady_k(L, w.accel_x, w.tau)
    L2 = make_porous_lattice(lb2d, w, "f32", stream, accel=2 * w.accel_x)
    k2, n2, ok2 = steady_k(L2, 2 * w.accel_x, w.tau)
    L2.close()
    return {"k_lu2": k1, "steps": n1, "converged": ok1, "k_at_twice_the_forcing": k2, "steps_2": n2,
            "darcy_rel_diff": (abs(k2 / k1 - 1) if ok1 and ok2 else None),
            "rule": "nu <u_x>_all / a_x, nu = (tau - 1/2)/3, once <u_x> changes by < 1e-6 over 1000 steps"}


def run_variant_storage(lb2d, torch, w, storage, steps, warmup, stream, rounding="nearest"):
    L = make_porous_lattice(lb2d, w, storage, stream, rounding)
    L.iteration(warmup)
    L.prepare(steps)
    ms = time_steps(torch, stream, L.iteration, steps)
    n = w.nx * w.ny
    nfl = L.budgets()["fluid_nodes"]
    per = ms / steps
    byt = nfl * 18 * STORE_BYTES[storage] + n
    out = {"mlups": n * steps / (ms * 1e-3) / 1e6, "ms_per_step": per,
           "algorithmic_GBps": byt / (per * 1e-3) / 1e9, "steps": steps}
    L.close()
    return out


def run_channel(lb2d, torch, stream, nx=128, ny=64, accel=1e-6, tau=1.0, steps=5000):
    """The plain channel in FP64 (128 x 64 nodes, walls at rows 0 and 63,
    g = 1e-6, tau = 1, from rest): MLUPS of the 5000-step start-up (its
    first 64 steps, which build the launch graph, untimed), its
    velocity profile against the start-up solution of the force-driven
    channel (Fourier series, walls half-way at y = 0.5 and ny - 1.5) and the
    mass drift.  A lattice this small is launch-bound, not HBM-bound."""
    import numpy as np
    L = lb2d.Lattice(0)
    L.lattice("d2q9", nx, ny, tau)
    L.boundary_style("noslip")
    L.obstacle_rect(0, nx - 1, 0, 0)
    L.obstacle_rect(0, nx - 1, ny - 1, ny - 1)
    L.aveacceleration(1, accel)
    L.bind("f64", stream=stream)
    m0 = L.budgets()["mass0"]
    L.iteration(GRAPH_WARMUP)
    timed = steps - GRAPH_WARMUP
    L.prepare(timed)
    ms = time_steps(torch, stream, L.iteration, timed)
    _, ux, _ = L.moments(0)
    nu = (tau - 0.5) / 3.0
    H = ny - 2.0
    y = np.arange(1, ny - 1, dtype=float)
    xi, eta = y - 0.5, y - (ny - 1) / 2.0
    u = accel / (2 * nu) * ((H / 2) ** 2 - eta ** 2)
    for k in range(1, 400, 2):
        u -= 4 * accel * H ** 2 / (nu * math.pi ** 3 * k ** 3) * np.sin(k * math.pi * xi / H) \
            * math.exp(-nu * k * k * math.pi ** 2 * steps / H ** 2)
    umax = accel * H * H / (8 * nu)
    out = {"workload": f"channel {nx}x{ny}, walls at rows 0 and {ny - 1}, g {accel}, tau {tau}, f64, from rest",
           "steps": steps, "timed_steps": timed, "mlups": nx * ny * timed / (ms * 1e-3) / 1e6,
           "ms_per_step": ms / timed,
           "u_err_vs_startup_series": float(np.abs(ux[1:-1, :] - u[:, None]).max() / umax),
           "mass_drift": (L.budgets()["mass0"] - m0) / m0}
    L.close()
    return out


def run_droplet(lb2d, torch, stream, storage):
    """The paper's parallelization example (351 x 201 nodes, two components,
    a droplet on a solid row): the 500 steps the paper times, on one GPU.
    The paper plots its CPU timings without numbers, so this is context, not
    a comparison.  A lattice this small is launch-bound."""
    from paper_1202_0442_amd import inputs
    w = inputs.parallel_droplet()
    e = w.extra
    L = lb2d.Lattice(0)
    L.lattice("d2q9", w.nx, w.ny, w.tau)
    L.fluids(w.tau, e["tau2"])
    L.boundary_style("noslip")
    for r in w.rects:
        L.obstacle_rect(*r)
    L.set_fields(0, e["rho"][0])
    L.set_fields(1, e["rho"][1])
    L.interforce(e["G"])
    L.adhesiveforce(e["Gads"][0], 0)
    L.adhesiveforce(e["Gads"][1], 1)
    L.bind(storage, stream=stream)
    L.iteration(GRAPH_WARMUP)
    L.prepare(w.steps)
    ms = time_steps(torch, stream, L.iteration, w.steps)
    out = {"workload": f"paper's parallelization droplet, {w.nx}x{w.ny}, two components, {storage}",
           "steps": w.steps, "warmup": GRAPH_WARMUP, "ms_total": ms, "ms_per_step": ms / w.steps,
           "mlups": w.nx * w.ny * w.steps / (ms * 1e-3) / 1e6}
    L.close()
    return out


def run_sc_solute(lb2d, torch, n, steps, warmup, stream, storage="f32", rounding="nearest"):
    from paper_1202_0442_amd import inputs
    w = inputs.sc_solute(n=n)
    e = w.extra
    rho_a, rho_b = inputs.sc_initial_fields(w)
    L = lb2d.Lattice(0)
    L.lattice("d2q9", w.nx, w.ny, w.tau)
    L.fluids(w.tau, e["tau2"])
    L.solute(e["tau_s"], 9)
    L.solute_opening("xlo", "dirichlet", e["C_in"])
    L.solute_opening("xhi", "adiabatic", 0.0)
    L.boundary_style("noslip")
    for (xc, yc, r) in w.discs:
        L.obstacle_circle(xc, yc, r)
    L.surface_reaction(e["kr"], e["Cs"], "growth", e["b0"], e["bmax"], e["rng_seed"])
    L.set_fields(0, rho_a.ravel())
    L.set_fields(1, rho_b.ravel())
    L.interforce(e["G"])
    L.adhesiveforce(e["Gads"][0], 0)
    L.adhesiveforce(e["Gads"][1], 1)
    L.rounding(rounding, 1)
    L.bind(storage, stream=stream)
    b0 = L.budgets()
    L.iteration(warmup)
    L.prepare(steps)
    ms = time_steps(torch, stream, L.iteration, steps)
    # step-kernel time alone (growth/tally kernel excluded), event-bracketed
    L.set_timing(True)
    L.iteration(20)
    kms, _ = L.kernel_time()
    L.set_timing(False)
    b = L.budgets()
    nn = w.nx * w.ny
    nfl = b["fluid_nodes"]
    # per fluid node: 2 comps + solute, 9 loads + 9 stores; mask 1 byte
    byt = nfl * 3 * 18 * STORE_BYTES[storage] + nn
    # budgets since bind: solute + deposit + solute removed by growth +
    # deposit consumed by growth - b0 per grown node + outflow - inflow is
    # conserved; each component's mass plus the mass removed by growth too
    sol = lambda d: (d["solute"] + d["deposit"] + d["removed_solute"] + d["consumed_deposit"]
                     - e["b0"] * d["grown_nodes"] + d["outflow"] - d["inflow"])
    out = {"workload": f"two-component Shan-Chen + D2Q9 solute + growth, {w.nx}x{w.ny}, {storage}, "
                       f"{rounding} rounding",
           "mlups": nn * steps / (ms * 1e-3) / 1e6, "ms_per_step": ms / steps,
           "step_kernel_ms": kms, "step_kernel_algorithmic_GBps": byt / (kms * 1e-3) / 1e9,
           "step_kernel_frac_hbm": byt / (kms * 1e-3) / 1e9 / PEAK_HBM_GBPS,
           "grown_nodes": b["grown_nodes"], "steps": warmup + steps + 20,
           "solute_budget_rel_err": abs(sol(b) - sol(b0)) / max(abs(b["inflow"]), abs(sol(b0)), 1e-300),
           "mass_rel_err": max(abs(b[f"mass{c}"] + b[f"removed_mass{c}"] - b0[f"mass{c}"]) / b0[f"mass{c}"]
                               for c in (0, 1))}
    L.close()
    return out


def run_phase(lb2d, torch, n, steps, warmup, stream, storage="f32"):
    """One-component Shan-Chen (psi form) phase separation, the paper's
    parameters on an n x n box: throughput of the general step with the
    psi density tile."""
    from paper_1202_0442_amd import inputs
    w = inputs.phase_separation(n=n)
    e = w.extra
    L = lb2d.Lattice(0)
    L.lattice("d2q9", w.nx, w.ny, w.tau)
    L.set_fields(0, e["rho"])
    L.interforce(e["G"], e["psi0"], e["rho0"])
    L.bind(storage, stream=stream)
    m0 = L.budgets()["mass0"]
    L.iteration(warmup)
    L.prepare(steps)
    ms = time_steps(torch, stream, L.iteration, steps)
    L.set_timing(True)
    L.iteration(20)
    kms, _ = L.kernel_time()
    L.set_timing(False)
    nn = w.nx * w.ny
    byt = nn * 73  # every node fluid: 9 loads + 9 stores of 4 bytes + link word
    rho, _, _ = L.moments(0)
    out = {"workload": f"one-component Shan-Chen phase separation {n}x{n} (G -120, psi0 4, rho0 200), {storage}",
           "mlups": nn * steps / (ms * 1e-3) / 1e6, "ms_per_step": ms / steps, "step_kernel_ms": kms,
           "step_kernel_algorithmic_GBps": byt / (kms * 1e-3) / 1e9,
           "step_kernel_frac_hbm": byt / (kms * 1e-3) / 1e9 / PEAK_HBM_GBPS,
           "rho_min": float(rho.min()), "rho_max": float(rho.max()),
           "mass_drift": L.budgets()["mass0"] / m0 - 1.0, "steps": steps + warmup + 20}
    L.close()
    return out


def run_growth_sweep(lb2d, torch, stream, storage="f64"):
    """The paper's surface-growth sweep, Da = 4, 20, 40, 80 at its full
    20 000 steps: grown nodes, perimeter per square root of area (larger =
    less compact), solute-budget closure and time."""
    import numpy as np
    from paper_1202_0442_amd import inputs
    out = {}
    for kr in (5e-3, 0.025, 0.05, 0.1):
        w = inputs.surface_growth(kr)
        e = w.extra
        L = lb2d.Lattice(0)
        L.lattice("d2q9", w.nx, w.ny, w.tau)
        L.solute(e["tau_s"], 4)
        L.boundary_style("noslip")
        for r in w.rects:
            L.obstacle_rect(*r)
        L.surface_reaction(e["kr"], e["Cs"], "growth", e["b0"], e["bmax"], e["rng_seed"])
        L.set_fields(0, np.full(w.nx * w.ny, w.rho0))
        L.set_concentration(np.full(w.nx * w.ny, e["C0"]))
        L.bind(storage, stream=stream)
        b0 = L.budgets()
        L.prepare(w.steps)
        ms = time_steps(torch, stream, L.iteration, w.steps)
        b1 = L.budgets()
        m = L.mask().astype(int)
        per = (np.abs(np.diff(m, axis=0, append=m[:1])).sum() + np.abs(np.diff(m, axis=1, append=m[:, :1])).sum())
        lhs = b1["solute"] + b1["deposit"] + b1["removed_solute"] + b1["consumed_deposit"] - e["b0"] * b1["grown_nodes"]
        rhs = b0["solute"] + b0["deposit"]
        out[f"Da{e['Da']:g}"] = {"kr": kr, "grown_nodes": b1["grown_nodes"],
                                 "perimeter_per_sqrt_area": float(per / np.sqrt(m.sum())),
                                 "solute_budget_rel_err": abs(lhs - rhs) / rhs, "ms": ms,
                                 "mlups": w.nx * w.ny * w.steps / (ms * 1e-3) / 1e6}
        L.close()
    return {"workload": "paper's surface growth: 200x200 periodic, 11x11 seed, D2Q4 solute C0 1.5, Cs 0.5, "
                        f"b0 0.5, bmax 1, tau = tau_s = 1, 20000 steps, {storage}", "sweep": out}


def run_ensemble(lb2d, torch, count, steps, seq_steps, stream, storage="f32", rounding="nearest"):
    from paper_1202_0442_amd import inputs
    ws = inputs.ensemble(count=count)
    lats = [make_porous_lattice(lb2d, w, storage, stream, rounding) for w in ws]
    ntot = sum(w.nx * w.ny for w in ws)
    # one lattice at a time with the one-fluid kernel: each lattice runs its
    # k steps (graph-launched: k is a multiple of the 60-step graph, built in
    # the warm-up) before the next one starts
    ms_seq = None
    if seq_steps:
        assert seq_steps % 60 == 0
        for L in lats:
            L.iteration(GRAPH_WARMUP)

        def seq(k):
            for L in lats:
                L.iteration(k)
        ms_seq = time_steps(torch, stream, seq, seq_steps)
    nfl = sum(L.budgets()["fluid_nodes"] for L in lats)
    B = lb2d.Batch(0)
    for L in lats:
        B.add(L)
    B.finalize(stream=stream)
    B.iteration(GRAPH_WARMUP)
    ms_b = time_steps(torch, stream, B.iteration, steps)
    # algorithmic bytes of one batched step: 18 values per fluid node of
    # every lattice and the 1-byte mask of every node; a launch advances
    # `spl` steps (5 for the multi-step tile)
    spl = B.steps_per_launch()
    step_bytes = nfl * 18 * STORE_BYTES[storage] + ntot
    byt = spl * step_bytes
    per = ms_b / steps
    launch_ms = per * spl
    trials = B.trials()
    spread = {}
    for t in trials:
        k = f"{t['tile_w']}x{t['tile_h']}"
        spread[k] = min(spread.get(k, 1e30), t["ms"])
    out = {"workload": f"{count} porous lattices, sides log-uniform 256..1536, {ntot} nodes, {storage}"
                       + ("" if rounding == "nearest" else f", {rounding} rounding"),
           "batched_mlups": ntot * steps / (ms_b * 1e-3) / 1e6,
           "sequential_mlups": ntot * seq_steps / (ms_seq * 1e-3) / 1e6 if seq_steps else None,
           "tuned": B.config(), "autotuner_trials": len(trials),
           "best_ms_per_tile_shape": {k: round(v, 4) for k, v in spread.items()},
           "roofline": {"bound": "hbm", "achieved": round(byt / (launch_ms * 1e-3) / 1e9, 1),
                        "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                        "frac": round(byt / (launch_ms * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4),
                        "kernel": "k_batch_ms" if spl > 1 else "k_batch", "steps_per_launch": spl,
                        "bytes_per_launch": byt, "launch_ms": launch_ms,
                        "bytes_rule": f"{18 * STORE_BYTES[storage]} B per fluid node of every lattice and step "
                                      f"+ 1 B mask per node and step, times the {spl} step(s) one launch "
                                      "advances"},
           "ms_per_step": per, "steps": steps, "sequential_steps": seq_steps}
    if spl > 1:
        out["roofline"]["launch_io_bytes"] = step_bytes
        out["roofline"]["launch_io_GBps"] = round(step_bytes / (launch_ms * 1e-3) / 1e9, 1)
    out["speedup"] = out["batched_mlups"] / out["sequential_mlups"] if seq_steps else None
    B.close()
    for L in lats:
        L.close()
    return out


def run_precision(lb2d, torch, stream, ref_path, n=2048, steps=10000):
    """Precision sweep: the channel and porous workloads at n x n, stored as
    FP32, FP16 and BF16 deviations (FP32 arithmetic), against the FP64
    oracle after `steps` steps: max and L2 errors of rho and u, MLUPS and
    algorithmic GB/s."""
    import numpy as np
    from paper_1202_0442_amd import inputs
    if ref_path and os.path.exists(ref_path):
        ref = dict(np.load(ref_path))
        assert int(ref["n"]) == n and int(ref["steps"]) == steps, "reference of another size"
    else:
        from oracle import reference_fields as rf
        log("computing the oracle reference (slow)")
        cr, cu, cv = rf.channel(n, steps)
        pr, pu, pv, pm = rf.porous(n, steps)
        ref = dict(channel_rho=cr, channel_ux=cu, channel_uy=cv, porous_rho=pr, porous_ux=pu,
                   porous_uy=pv, porous_mask=pm)
    res = {}
    for wl in ("channel", "porous"):
        if wl == "channel":
            w = inputs.poiseuille(nx=n, ny=n, accel=1e-6, tau=1.0)
            rr = np.broadcast_to(ref["channel_rho"][:, None], (n, n))
            ru = np.broadcast_to(ref["channel_ux"][:, None], (n, n))
            rv = np.broadcast_to(ref["channel_uy"][:, None], (n, n))
        else:
            w = inputs.porous(n=n, seed=4)
            rr, ru, rv = ref["porous_rho"], ref["porous_ux"], ref["porous_uy"]
        fl = rr != -11.0
        for key in ("f32", "f16", "bf16", "f16sr", "bf16sr"):
            st = key[:-2] if key.endswith("sr") else key
            L = make_porous_lattice(lb2d, w, st, stream, "stochastic" if key.endswith("sr") else "nearest")
            nfl = L.budgets()["fluid_nodes"]
            ms = time_steps(torch, stream, L.iteration, steps)
            g_r, g_u, g_v = L.moments(0)
            assert np.array_equal(g_r == -11.0, ~fl)
            du = np.hypot(g_u - ru, g_v - rv)[fl]
            um = np.hypot(ru, rv)[fl]
            drho = np.abs(g_r - rr)[fl]
            per = ms / steps
            res[f"{wl}_{key}"] = {
                "u_max_rel": float(du.max() / um.max()),
                "u_l2_rel": float(np.sqrt((du ** 2).sum() / (um ** 2).sum())),
                "rho_max_abs": float(drho.max()),
                "rho_l2_abs": float(np.sqrt((drho ** 2).mean())),
                "mlups": n * n / (per * 1e-3) / 1e6,
                "algorithmic_GBps": (nfl * 18 * STORE_BYTES[st] + n * n) / (per * 1e-3) / 1e9,
            }
            log(f"precision {wl} {key}: {res[f'{wl}_{key}']}")
            L.close()
            torch.cuda.empty_cache()
    return {"precision_sweep": res, "n": n, "steps": steps,
            "reference": "FP64 oracle (channel: 4-wide strip, uniform in x; porous: full lattice)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=4096, help="lattice side")
    ap.add_argument("--workload", default="porous", choices=("porous", "channel"),
                    help="porous: discs r 8..24 to porosity 0.6; channel: walls at rows 0 and n-1, a_x 1e-6, tau 1")
    ap.add_argument("--seed", type=int, default=2, help="seed of the porous geometry")
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--variants", default="all",
                    help="all | none | comma list of f16,bf16,sc,phase,growth,batch,channel,droplet")
    ap.add_argument("--rounding", default="nearest", choices=("nearest", "stochastic"),
                    help="rounding of 16-bit storage in the --no-main two-component + solute run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-readout", action="store_true")
    ap.add_argument("--no-permeability", action="store_true",
                    help="skip the steady-state permeability runs after the timed steps")
    ap.add_argument("--sc-steps", type=int, default=20000,
                    help="steps of the two-component, phase and ensemble variants run with --no-main; "
                         "the two-component variant's configuration runs 20000")
    ap.add_argument("--no-sequential", action="store_true",
                    help="with --no-main: the ensemble without its one-at-a-time baseline")
    ap.add_argument("--no-main", action="store_true",
                    help="profiling aid: run only the selected variants (no headline line)")
    ap.add_argument("--precision", action="store_true",
                    help="run the precision sweep instead (prints its own JSON line)")
    ap.add_argument("--precision-ref", default="refdata/precision_2048.npz",
                    help="npz written by `python -m oracle.reference_fields` (else computed here)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs on one GPU; --gpus must be 1 "
              "(several GPUs would shard the lattice in y slabs, which is not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1202_0442_amd import inputs, lb2d
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    stream = torch.cuda.Stream()
    if args.precision:
        print(json.dumps(run_precision(lb2d, torch, stream, os.path.join(ROOT, args.precision_ref))), flush=True)
        return
    if args.no_main:
        want = set(args.variants.split(",")) if args.variants not in ("all", "none") else set()
        res = {}
        if "sc" in want:
            res["sc_solute"] = run_sc_solute(lb2d, torch, 2048, args.sc_steps, 10, stream, storage=args.storage,
                                             rounding=args.rounding)
        if "phase" in want:
            res["phase"] = run_phase(lb2d, torch, 4096, args.sc_steps, 10, stream)
        if "growth" in want:
            res["growth"] = run_growth_sweep(lb2d, torch, stream)
        if "batch" in want:
            res["ensemble"] = run_ensemble(lb2d, torch, 256, args.sc_steps, 0 if args.no_sequential else 120,
                                           stream, storage=args.storage)
        if "channel" in want:
            res["channel"] = run_channel(lb2d, torch, stream)
        if "droplet" in want:
            for st in ("f64", "f32"):
                res[f"droplet_{st}"] = run_droplet(lb2d, torch, stream, st)
        print(json.dumps(res), flush=True)
        lb2d.copy_bench(1 << 30, reps=3, stream=stream)
        return
    log(f"generating {args.workload} workload")
    if args.workload == "porous":
        w = inputs.porous(n=args.n, seed=args.seed)
        wname = f"porous {w.nx}x{w.ny}, non-overlapping discs r 8..24, porosity 0.6, periodic, tau 0.8, accel 1e-5 (e1)"
        pname = f"porous{args.n}" + ("" if args.seed == 2 else f"_seed{args.seed}")
    else:
        w = inputs.poiseuille(nx=args.n, ny=args.n, accel=1e-6, tau=1.0)
        wname = f"channel {w.nx}x{w.ny}, walls at rows 0 and {w.ny - 1}, periodic x, tau 1, accel 1e-6 (e1)"
        pname = f"channel{args.n}"
    L = make_porous_lattice(lb2d, w, args.storage, stream)
    n = w.nx * w.ny
    bud = L.budgets()
    nfl = int(bud["fluid_nodes"])
    log(f"lattice {w.nx}x{w.ny}, fluid fraction {nfl / n:.4f}; warmup {args.warmup}")
    L.iteration(args.warmup)
    L.prepare(args.steps)        # capture the launch graphs outside the timed region
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    ms = time_steps(torch, stream, L.iteration, args.steps)
    per = ms / args.steps
    mlups = n * args.steps / (ms * 1e-3) / 1e6
    log(f"{mlups:.0f} MLUPS, {per * 1e3:.1f} us/step")
    # the dominant kernel advances `spl` steps per launch (the multi-step
    # kernel: 5), launched back to back inside the graphs: launch time =
    # spl x step time (HIP events on the stream the kernel runs on)
    spl = L.steps_per_launch()
    kernel = "k_plain_ms" if spl > 1 else "k_plain"
    launch_ms = per * spl
    step_bytes = nfl * 18 * STORE_BYTES[args.storage] + n
    bytes_launch = spl * step_bytes
    achieved = bytes_launch / (launch_ms * 1e-3) / 1e9
    traffic = measured_traffic(f"{kernel}_{args.storage}_{pname}.md")
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": per,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.storage, "data": "synthetic",
        "config": {"workload": f"{wname}, {args.storage} shifted storage",
                   "nx": w.nx, "ny": w.ny, "discs": len(w.discs), "fluid_fraction": nfl / n},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": traffic,
                     "kernel": kernel, "steps_per_launch": spl, "bytes_per_launch": bytes_launch,
                     "launch_ms": launch_ms,
                     "bytes_rule": f"{18 * STORE_BYTES[args.storage]} B per fluid node and step (9 loads + 9 stores "
                                   f"of {STORE_BYTES[args.storage]} B) + 1 B mask per node and step, times the "
                                   f"{spl} step(s) one launch advances"},
        "mflups": round(nfl * args.steps / (ms * 1e-3) / 1e6, 1),
    }
    # dense accounting (every node, solids included, moves 18 values + mask):
    # the bandwidth a kernel without obstacle skipping would need for the
    # same MLUPS; the kernel itself moves only fluid-bearing lines
    dense = n * (18 * STORE_BYTES[args.storage] + 1) / (per * 1e-3) / 1e9
    out["roofline"]["dense_equiv_GBps"] = round(dense, 1)
    out["roofline"]["dense_equiv_frac"] = round(dense / PEAK_HBM_GBPS, 4)
    if spl > 1:
        # what a multi-step launch must move at least: every fluid population
        # read once and written once, and the mask (the first steps' values
        # stay in LDS), at the launch's duration
        out["roofline"]["launch_io_bytes"] = step_bytes
        out["roofline"]["launch_io_GBps"] = round(step_bytes / (launch_ms * 1e-3) / 1e9, 1)
        out["roofline"]["launch_io_frac"] = round(step_bytes / (launch_ms * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4)
    if traffic is not None:
        # measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE,
        # scaled by a copy kernel of known size) at this launch's duration
        out["roofline"]["traffic_GBps"] = round(traffic / (launch_ms * 1e-3) / 1e9, 1)
        out["roofline"]["traffic_frac"] = round(traffic / (launch_ms * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4)
    mass_drift = None
    if not args.no_readout:
        b1 = L.budgets()
        mass_drift = (b1["mass0"] - bud["mass0"]) / bud["mass0"]
        out["mass_drift"] = mass_drift
        if not args.no_permeability and args.workload == "porous":
            log("permeability: continuing to steady state, then at twice the forcing")
            out["permeability"] = permeability(lb2d, w, L, stream)
    L.close()
    torch.cuda.empty_cache()

    log("copy ceiling")
    cb = 1 << 30
    cms = lb2d.copy_bench(cb, reps=20, stream=stream)
    out["copy_ceiling_GBps"] = round(2 * cb / (cms * 1e-3) / 1e9, 1)
    out["roofline"]["frac_of_copy"] = round(achieved / out["copy_ceiling_GBps"], 4)
    if spl > 1:
        out["roofline"]["launch_io_frac_of_copy"] = round(out["roofline"]["launch_io_GBps"]
                                                          / out["copy_ceiling_GBps"], 4)

    want = set() if args.variants == "none" else (
        {"f16", "bf16", "sc", "phase", "growth", "batch", "channel", "droplet"} if args.variants == "all"
        else set(args.variants.split(",")))
    variants = {}
    for st in ("f16", "bf16"):
        if st in want:
            for rnd in ("nearest", "stochastic"):
                key = f"{st}_store" if rnd == "nearest" else f"{st}_store_stochastic"
                log(f"variant {key}")
                variants[key] = run_variant_storage(lb2d, torch, w, st, max(500, args.steps // 5), 50, stream,
                                                    rnd)
                variants[key]["speedup_vs_f32"] = variants[key]["mlups"] / mlups
                torch.cuda.empty_cache()
    if "sc" in want:
        log("variant two-component + solute 2048^2")
        variants["sc_solute"] = run_sc_solute(lb2d, torch, 2048, args.sc_steps, GRAPH_WARMUP, stream)
        torch.cuda.empty_cache()
        for st in ("f16", "bf16"):
            for rnd in ("nearest", "stochastic"):
                log(f"variant two-component + solute 2048^2, {st} storage, {rnd} rounding")
                key = f"sc_solute_{st}" + ("_sr" if rnd == "stochastic" else "")
                variants[key] = run_sc_solute(lb2d, torch, 2048, args.sc_steps, GRAPH_WARMUP, stream,
                                              storage=st, rounding=rnd)
                variants[key]["speedup_vs_f32"] = variants[key]["mlups"] / variants["sc_solute"]["mlups"]
                torch.cuda.empty_cache()
    if "phase" in want:
        log("variant one-component Shan-Chen 4096^2")
        variants["phase"] = run_phase(lb2d, torch, 4096, args.sc_steps, GRAPH_WARMUP, stream)
        torch.cuda.empty_cache()
    if "growth" in want:
        log("variant surface-growth sweep")
        variants["growth"] = run_growth_sweep(lb2d, torch, stream)
        torch.cuda.empty_cache()
    if "channel" in want:
        log("variant channel 128x64 f64")
        variants["channel"] = run_channel(lb2d, torch, stream)
    if "droplet" in want:
        log("variant the paper's parallelization droplet")
        for st in ("f64", "f32"):
            variants[f"droplet_{st}"] = run_droplet(lb2d, torch, stream, st)
    if "batch" in want:
        log("variant batched ensemble")
        variants["ensemble"] = run_ensemble(lb2d, torch, 256, 500, 120, stream)
        torch.cuda.empty_cache()
        log("variant batched ensemble, FP16 storage")
        variants["ensemble_f16"] = run_ensemble(lb2d, torch, 256, 500, 120, stream, storage="f16")
        variants["ensemble_f16"]["speedup_vs_f32_batched"] = (variants["ensemble_f16"]["batched_mlups"]
                                                             / variants["ensemble"]["batched_mlups"])
        torch.cuda.empty_cache()
        log("variant batched ensemble, FP16 storage, stochastic rounding")
        variants["ensemble_f16_sr"] = run_ensemble(lb2d, torch, 256, 500, 120, stream, storage="f16",
                                                   rounding="stochastic")
        variants["ensemble_f16_sr"]["speedup_vs_f32_batched"] = (variants["ensemble_f16_sr"]["batched_mlups"]
                                                                / variants["ensemble"]["batched_mlups"])
        torch.cuda.empty_cache()
    if variants:
        out["variants"] = variants
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
