#!/usr/bin/env python3
"""Throughput of the two-beam FFT BPM march on one MI355X.

One "step" = one pass of the whole hot path over one batch: every solve of the
workload marched through all of its z-steps (plan tables already built, entrance
envelopes already resident in HBM).  Default workload: the Laue bent-crystal
case, Nx = 16384, Nz = 8000, dz = 0.025 um, bend radii R = 1, 0.1, 10 m, FP32,
85 seeded Gaussian beams per radius (255 solves, one per compute unit).

After the headline it reports, as side legs, one FP64 flat-Bragg solve alone,
the 64-angle scan (and the scan replicated to 256 solves), the headline batch
in FP64, the dislocation batch (Nx 32768), the pulse-component batch (mixed
sizes, one launch), the paper's 3D case, the rows after the first-order march
and the serving mix (p50/p99 latency), and the FP64 oracle on the host.

Prints one JSON line (metric, value, roofline, cpu_baseline, legs, ...).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BPM cell-steps/s (Nx·Nz·2 beams), FP32 batched vs FP64 plain; p50/p99 solve ms"
# MI355X published vector peaks (TFLOP/s): FP32 157.3 (packed FP32 issue), FP64 78.6.
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
# The library is built without packed-FP32 instructions: one wave64 FP32 FMA
# per SIMD per 4 clocks, 256 CUs x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz.  This
# issue ceiling is reported beside the published peak, never in its place.
NONPACKED_F32_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


# the sources the march kernels are compiled from (device code and the
# descriptors it reads); host-side changes do not invalidate a profile
KERNEL_SOURCES = ("bpm_internal.hpp", "bpm_march.hpp", "bpm_march_kernels.hpp")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2601_06340_amd", "csrc")
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def workload(name: str, beams_per_radius: int, nz_override: int | None):
    from paper_2601_06340_amd import synth
    if name == "bent_laue":
        kw = {} if nz_override is None else {"nz": nz_override}
        cases = synth.bent_laue(radii_m=(1.0, 0.1, 10.0), beams_per_radius=beams_per_radius,
                                precision="f32", **kw)
        cfg = {"workload": "bent_laue", "nx": 16384, "nz": cases[0][0]["nz"], "dz_um": 0.025,
               "radii_m": [1.0, 0.1, 10.0], "beams_per_radius": beams_per_radius,
               "solves": len(cases), "precision": "f32"}
    elif name == "flat_bragg":
        kw = {} if nz_override is None else {"nz": nz_override}
        cases = synth.flat_bragg_scan(n_angles=64, precision="f64", **kw)
        cfg = {"workload": "flat_bragg", "nx": 4096, "nz": cases[0][0]["nz"], "angles": 64,
               "solves": 64, "precision": "f64"}
    elif name == "td_batch":
        cases = synth.td_batch()
        cfg = {"workload": "td_batch", "components": len(cases), "nx": "2048..16384",
               "nz": "1000..8000", "solves": len(cases), "precision": "f32"}
    else:
        raise SystemExit("unknown workload " + name)
    return cases, cfg


def time_batch(bpm, torch, cases, steps, warmup, keep=()):
    """Times `steps` batch launches; also returns the exit envelopes of the
    solves listed in `keep` (read back after the timed region)."""
    plans = [bpm.Plan(p) for p, _ in cases]
    batch = bpm.Batch(plans)
    d_in = batch.pack([(psi, None) for _, psi in cases])
    d_out = torch.empty_like(d_in)
    rt = torch.zeros(2 * len(plans), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    sid = stream.cuda_stream
    for _ in range(warmup):
        batch.run(d_in.data_ptr(), d_out.data_ptr(), rt.data_ptr(), sid)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(steps):
        batch.run(d_in.data_ptr(), d_out.data_ptr(), rt.data_ptr(), sid)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    total_ms = ev[0].elapsed_time(ev[steps])
    Rs = rt.cpu().numpy()
    kept = {}
    if keep:
        outs = batch.unpack(d_out)
        kept = {i: outs[i] for i in keep}
    batch.close()
    for p in plans:
        p.close()
    return per, total_ms, wall, Rs, kept


def fp32_error_vs_fp64(bpm, cases, Rs, kept):
    """The FP32 batch's error against FP64 marches of the same solves on the
    GPU (relative L2 over both envelopes, |dR|, |dT|)."""
    import numpy as np
    rows = []
    for i, (gp, gm) in sorted(kept.items()):
        p, psi = cases[i]
        plan = bpm.Plan(dict(p, precision="f64"))
        fp, fm, fR, fT = plan.propagate(psi)
        plan.close()
        d = np.concatenate([np.ravel(gp) - np.ravel(fp), np.ravel(gm) - np.ravel(fm)])
        ref = np.concatenate([np.ravel(fp), np.ravel(fm)])
        rows.append({"solve": i, "rel_l2": float(np.linalg.norm(d) / np.linalg.norm(ref)),
                     "dR": float(abs(Rs[2 * i] - fR)), "dT": float(abs(Rs[2 * i + 1] - fT))})
    return {"solves": rows, "rel_l2_max": max(r["rel_l2"] for r in rows),
            "dR_max": max(r["dR"] for r in rows), "dT_max": max(r["dT"] for r in rows),
            "what": "FP32 batch results against FP64 marches of the same solves on the GPU"}


def time_single(bpm, torch, case, steps, warmup):
    """One solve through the single-solve entry point (bpm_propagate_device):
    staged sizes and 3D envelopes spread over the whole device."""
    p, psi = case
    plan = bpm.Plan(p)
    one = bpm.Batch([plan])   # packs the entrance state
    d_in = one.pack([(psi, None)])
    d_out = torch.empty_like(d_in)
    rt = torch.zeros(2, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    sid = stream.cuda_stream
    for _ in range(warmup):
        plan.propagate_device(d_in.data_ptr(), d_out.data_ptr(), rt.data_ptr(), sid)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for k in range(steps):
        plan.propagate_device(d_in.data_ptr(), d_out.data_ptr(), rt.data_ptr(), sid)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    one.close()
    plan.close()
    ms = sum(per) / len(per)
    return {"ms": ms, "value": cell_steps(p) / (ms / 1e3)}


def fp64_plain(bpm, torch, synth):
    """One FP64 solve alone on the GPU (the flat Bragg case: Nx 4096, Nz 2000)."""
    p, psi = synth.flat_bragg_scan(n_angles=1, precision="f64")[0]
    per, total, _, _, _ = time_batch(bpm, torch, [(p, psi)], 3, 1)
    cs = cell_steps(p)
    return {"value": cs / (sum(per) / len(per) / 1e3), "unit": "cell-steps/s",
            "workload": "flat_bragg Nx 4096 Nz 2000, one FP64 solve", "ms": sum(per) / len(per)}


def flops(p) -> float:
    """Algorithmic flops of one solve: 10 log2(Nx) + 26 per cell-step (two
    complex FFTs of 5 N log2 N, the propagator 6, the coupling 14, a+-e^{+-i phi} 6)."""
    n = p["nx"] * max(1, int(p.get("ny", 1)))
    return (10 * math.log2(n) + 26) * cell_steps(p)


def alu_roofline(cases, ms, prec):
    """ALU roofline of one batch launch of `ms` milliseconds: achieved
    algorithmic TFLOP/s against the published vector peak of its precision,
    and (FP32) against the non-packed issue ceiling of this build."""
    fl = sum(flops(p) for p, _ in cases)
    achieved = fl / (ms / 1e3) / 1e12
    out = {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
           "frac": achieved / PEAK_TFLOPS[prec], "flop_per_cell_step": fl / sum(cell_steps(p) for p, _ in cases)}
    if prec == "f32":
        out["issue_ceiling"] = {"peak": NONPACKED_F32_TFLOPS, "frac": achieved / NONPACKED_F32_TFLOPS,
                                "what": "non-packed FP32 VALU issue rate (this build has no packed FP32 "
                                        "instructions): the ceiling the kernel can reach"}
    return out


def cell_steps(p) -> float:
    """Cells times z-steps of one solve, both beams (nx ny nz, ny = 1 in 2D)."""
    return 2.0 * p["nx"] * max(1, int(p.get("ny", 1))) * p["nz"]


def leg_batch(bpm, torch, cases, label, steps=1, warmup=1, keep=()):
    """Throughput of one workload batch in one launch per step; the solves in
    `keep` (FP32) are also compared with FP64 marches of the same solves."""
    print("leg %s: %d solves" % (label, len(cases)), file=sys.stderr, flush=True)
    per, total, _, Rs, kept = time_batch(bpm, torch, cases, steps, warmup, keep)
    cs = sum(cell_steps(p) for p, _ in cases)
    ms = total / steps
    out = {"value": cs / (ms / 1e3), "unit": "cell-steps/s", "ms_per_step": ms, "solves": len(cases),
           "cell_steps": cs}
    if kept:
        out["fp32_error_vs_fp64"] = fp32_error_vs_fp64(bpm, cases, Rs, kept)
    return out


def leg_next(bpm, torch, synth):
    """The rows after the first-order march: splitting orders 2 and 4
    (Eq. (13)) against order 1 on the 64-angle FP32 scan; the time-domain
    assembly of a 1024-component pulse on one grid; far-field propagation."""
    import numpy as np
    out = {}
    base = synth.flat_bragg_scan(n_angles=64, precision="f32")
    orders = {}
    for order in (1, 2, 4):
        cases = [(dict(p, split_order=order), psi) for p, psi in base]
        r = leg_batch(bpm, torch, cases, "split order %d" % order, steps=3, warmup=1)
        orders[str(order)] = {"ms": r["ms_per_step"], "value": r["value"]}
    out["split_orders"] = dict(orders, unit="cell-steps/s (z-steps of the scan, both beams)",
                               workload="64-angle FP32 scan, Nx 4096, Nz 2000, one batch launch per order")
    cases = synth.td_batch(n_comp=1024, nx_choices=(4096,), nz_range=(1000, 8000))
    print("leg td assembly: %d components" % len(cases), file=sys.stderr, flush=True)
    plans = [bpm.Plan(p) for p, _ in cases]
    batch = bpm.Batch(plans)
    buf = batch.pack([(psi, None) for _, psi in cases])
    stream = torch.cuda.current_stream()
    sid = stream.cuda_stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    batch.run(buf.data_ptr(), buf.data_ptr(), None, sid)        # warm-up march (plans, tables, code)
    batch.td_assemble(buf.data_ptr(), sid)
    buf = batch.pack([(psi, None) for _, psi in cases])
    torch.cuda.synchronize()
    ev[0].record(stream)
    batch.run(buf.data_ptr(), buf.data_ptr(), None, sid)
    ev[1].record(stream)
    batch.td_assemble(buf.data_ptr(), sid)
    ev[2].record(stream)
    torch.cuda.synchronize()
    cs = sum(cell_steps(p) for p, _ in cases)
    out["td_pulse"] = {"workload": "1024 components of a 20 fs pulse on one grid, Nx 4096, Nz 1000-8000, FP32: "
                                   "one batch march, then bpm_td_assemble to a [2][4096][1024] time trace",
                       "march_ms": ev[0].elapsed_time(ev[1]), "march_value": cs / (ev[0].elapsed_time(ev[1]) / 1e3),
                       "assemble_ms": ev[1].elapsed_time(ev[2]), "unit": "cell-steps/s"}
    batch.close()
    for pl in plans:
        pl.close()
    ff = {}
    for nx in (16384, 65536):
        p, psi = synth.flat_bragg_scan(n_angles=1, nx=nx, nz=10, precision="f32")[0]
        plan = bpm.Plan(p)
        st = torch.zeros(2 * nx, dtype=torch.complex64, device="cuda")
        st[:nx] = torch.from_numpy(psi.astype(np.complex64)).cuda()
        dst = torch.empty_like(st)
        plan.far_field_device(2.0e6, st.data_ptr(), dst.data_ptr(), sid)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(100):
            plan.far_field_device(2.0e6, st.data_ptr(), dst.data_ptr(), sid)
        e1.record(stream)
        torch.cuda.synchronize()
        ff[str(nx)] = e0.elapsed_time(e1) / 100
        plan.close()
    out["far_field_ms"] = dict(ff, what="one bpm_far_field call (2 m of vacuum, both beams), FP32, by nx")
    return out


def leg_serve(bpm, synth, n_req, rate_hz, budget_gb, chunk_steps):
    """Serving mix: a seeded Poisson stream submitted in real time to the
    continuous-batching server; latency = submit -> done on the server clock."""
    reqs = synth.serve_mix(n_req=n_req, rate_hz=rate_hz)
    print("leg serving: %d requests at %.0f/s" % (n_req, rate_hz), file=sys.stderr, flush=True)
    srv = bpm.Server(hbm_budget_bytes=int(budget_gb * (1 << 30)), max_slots=1024, chunk_steps=chunk_steps)
    t0 = time.perf_counter()
    tickets = []
    trace = []   # (seconds since the first arrival, cell-steps done, solves in flight), about once a second

    def sample():
        st = srv.stats()
        trace.append((time.perf_counter() - t0, st["cell_steps_done"],
                      st["admitted"] - st["completed"] - st["cancelled"] - st["failed"]))

    for r in reqs:
        dt = t0 + r["t_arrival"] - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        tickets.append(srv.submit(r["problem"], r["psi_p0"], want_fields=False))
        if not trace or time.perf_counter() - t0 - trace[-1][0] >= 1.0:
            sample()
    sample()
    drained = srv.drain(900.0)
    res = [srv.poll(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    good = [(r, x) for r, x in zip(reqs, res) if x is not None and x["status"] == 0]
    lat = sorted((x["t_done"] - x["t_submit"]) * 1e3 for _, x in good)

    def q(v, f):
        return v[min(len(v) - 1, max(0, int(math.ceil(f * len(v))) - 1))] if v else None

    span = max(x["t_done"] for _, x in good) - min(x["t_submit"] for _, x in good) if good else 0.0
    cs = sum(cell_steps(r) for r, _ in good)
    # steady state: the rate at which the server completed cell-steps while
    # requests kept arriving, after a ramp of 10 s (least-squares slope)
    win = [(t, c, a) for t, c, a in trace if 10.0 <= t <= reqs[-1]["t_arrival"]]
    steady = None
    if len(win) >= 5:
        ts = [w[0] for w in win]
        cs_t = [w[1] for w in win]
        tm, cm = sum(ts) / len(ts), sum(cs_t) / len(cs_t)
        steady = (sum((a - tm) * (b - cm) for a, b in zip(ts, cs_t)) / sum((a - tm) ** 2 for a in ts))
    return {"requests": n_req, "completed": len(good), "drained": bool(drained), "rate_hz": rate_hz,
            "p50_ms": q(lat, 0.5), "p99_ms": q(lat, 0.99), "max_ms": lat[-1] if lat else None,
            "value": cs / span if span > 0 else None, "unit": "cell-steps/s",
            "steady_state_value": steady,
            "in_flight_during_arrivals": [round(a) for _, _, a in trace[::5]],
            "value_what": "all completed cell-steps over first submit to last completion (includes the drain "
                          "of the last large requests after arrivals end); steady_state_value: the completion "
                          "rate while requests arrive, from 10 s to the last arrival",
            "offered": sum(cell_steps(r) for r in reqs) / reqs[-1]["t_arrival"],
            "launches": stats["launches"], "wide_lane_solves": stats["wide"], "peak_bytes": stats["peak_bytes"],
            "rounds": stats.get("rounds"),
            "active_max": stats.get("active_max"), "worker_device_wait_s": stats.get("t_device_wait_s"),
            "worker_host_s": stats.get("t_host_s"),
            "chunk_steps": chunk_steps,
            "budget_gb": budget_gb}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> dict:
    """Cores this process may run on, and the share it uses: a one-GPU share of
    the host is 16 cores, whatever the machine's total."""
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    return {"machine": os.cpu_count() or 1, "allowed": allowed, "used": max(1, min(16, allowed))}


def cpu_baseline(cases, target_s=12.0):
    """The FP64 oracle on the host cores over a bounded sample of the workload."""
    import oracle
    hc = host_cores()
    cores = hc["used"]
    nsolve = min(cores, len(cases))   # one solve per thread
    # size the sample: time one short solve first
    p0, psi0 = cases[0]
    probe = dict(p0, nz=20, seg=p0["seg"][:20])
    t = time.perf_counter()
    oracle.propagate(probe, psi0)
    per_step = (time.perf_counter() - t) / 20
    nz = max(20, min(p0["nz"], int(target_s / per_step)))
    sample = []
    for p, psi in cases[:nsolve]:
        q = dict(p, nz=nz, seg=p["seg"][:nz])
        if isinstance(q.get("strain"), dict) and q["strain"].get("kind") == "table":
            q["strain"] = dict(q["strain"], u_table=q["strain"]["u_table"][:nz])
        sample.append((q, psi))
    t = time.perf_counter()
    oracle.propagate_batch([q for q, _ in sample], [(psi, None) for _, psi in sample], nthreads=cores)
    wall = time.perf_counter() - t
    cs = sum(cell_steps(q) for q, _ in sample)
    return {"value": cs / wall, "unit": "cell-steps/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cores": hc,
            "sample": "%d of the %d solves, first %d of %d z-steps each, one solve per thread on %d threads "
                      "(%.1f s wall)" % (nsolve, len(cases), nz, p0["nz"], cores, wall)}


def traffic_entry(kernel: str, launch_cell_steps: float):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d.get(kernel)
        if not e or e.get("source_hash") != kernel_source_hash():
            return None
        return (e["fetch_bytes_per_cell_step"] + e["write_bytes_per_cell_step"]) * launch_cell_steps
    except (ValueError, KeyError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="bent_laue", choices=["bent_laue", "flat_bragg", "td_batch"])
    ap.add_argument("--beams-per-radius", type=int, default=85)
    ap.add_argument("--nz", type=int, default=None, help="shorter march (profiling runs only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-plain", action="store_true")
    ap.add_argument("--legs", default="cfg0,cfg0x4,cfg1f64,cfg2,cfg3,3d,next,cfg4",
                    help="extra workloads after the headline: cfg0 (64-angle FP64 scan, and its FP32 "
                         "twin), cfg0x4 (the scan replicated to 256 solves), cfg1f64 (the headline batch "
                         "in FP64), cfg2 (dislocation, Nx 32768), cfg3 (pulse "
                         "components, one mixed launch), 3d (the paper's 3D case), cfg4 (serving mix); "
                         "'none' for the headline only")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-chunk", type=int, default=256)
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the schedule autotuner for the headline size (64 synthetic solves, 100 steps)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="first run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only. Every solve is independent, so N GPUs would each march "
              "their own share of the batch (split by cell-step cost) and gather R/T at the end; "
              "no multi-GPU figure is taken here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2601_06340_amd import bpm, synth
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if not os.path.exists(bpm.LIB_PATH):
        from paper_2601_06340_amd import build as b
        b.build()

    if args.copy_calibration_mb:
        # a plain elementwise kernel (torch.neg) that reads and writes nb bytes
        # once each: the scale for the FETCH_SIZE / WRITE_SIZE counters
        nb = args.copy_calibration_mb << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print("copy calibration: torch.neg, %d bytes read + %d bytes written per launch" % (nb, nb),
              file=sys.stderr)
    cases, cfg = workload(args.workload, args.beams_per_radius, args.nz)
    nx = cases[0][0]["nx"]
    uniform = all(p["nx"] == nx for p, _ in cases)
    prec = cases[0][0]["precision"]
    tuned = None
    if uniform and not args.no_autotune:
        # the batch below takes the kernel family the autotuner measures fastest
        kind = bpm.STRAIN[(cases[0][0].get("strain") or {}).get("kind", "none")]
        if all(bpm.STRAIN[(p.get("strain") or {}).get("kind", "none")] == kind for p, _ in cases):
            print("autotune %s nx %d" % (prec, nx), file=sys.stderr, flush=True)
            tuned = bpm.autotune(prec, nx, kind, nsolves=64, nsteps=100)
    print("workload %s: %d solves" % (cfg["workload"], len(cases)), file=sys.stderr, flush=True)
    launch_cs = sum(cell_steps(p) for p, _ in cases)
    keep = sorted({0, len(cases) // 2, len(cases) - 1}) if prec == "f32" else []
    per, total_ms, wall, Rs, kept = time_batch(bpm, torch, cases, args.steps, args.warmup, keep)
    ms = total_ms / args.steps
    value = launch_cs / (ms / 1e3)
    per_sorted = sorted(per)

    def pct(q):
        k = min(len(per_sorted) - 1, max(0, int(math.ceil(q * len(per_sorted))) - 1))
        return per_sorted[k]

    tname = "float" if prec == "f32" else "double"
    sched = tuned["schedule"] if tuned else "uniform"
    if not uniform or sched == "mixed":
        kernel = "k_march_mixed<%s>" % tname
    elif sched == "any":
        kernel = "k_march_any<%s>" % tname
    else:
        # the per-size kernel's strain class (template argument): 0 none,
        # 1 polynomial, 2 dislocation / table, 3 polynomial without X^2
        def strain_cls(pr):
            st = pr.get("strain") or {"kind": "none"}
            if st.get("kind", "none") == "none":
                return 0
            if st["kind"] == "poly2":
                return 3 if float(st["c"][3]) == 0.0 else 1
            return 2
        classes = {strain_cls(pr) for pr, _ in cases}
        kernel = "k_march_uniform<%s,%d%s>" % (tname, int(math.log2(nx)),
                                               ",%d" % classes.pop() if len(classes) == 1 else "")
    roof = alu_roofline(cases, sum(per) / len(per), prec)
    roof.update(traffic=traffic_entry(kernel, launch_cs), kernel=kernel)

    out = {"metric": METRIC, "value": value, "unit": "cell-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": prec, "data": "synthetic", "config": cfg,
           "latency_ms": {"p50": pct(0.5), "p99": pct(0.99), "what": "batch completion per step"},
           "roofline": roof, "wall_s": wall}
    if tuned:
        out["autotune"] = dict(tuned, what="kernel family of the headline batch, timed on 64 synthetic "
                                           "solves of its size and strain kind (ms per 100-step batch march)")
    if not args.no_fp64_plain:
        out["fp64_plain"] = fp64_plain(bpm, torch, synth)
        out["fp32_batched_over_fp64_plain"] = value / out["fp64_plain"]["value"]
        out["fp32_batched_over_fp64_plain_what"] = (
            "headline FP32 batch (255 solves on 255 CUs) over one FP64 solve alone on one CU: a batching "
            "ratio; legs.cfg1_fp64_batch gives FP32 over FP64 at equal batching")
    out["R_mean"] = float(np.mean(Rs[0::2]))
    if kept:
        out["fp32_error_vs_fp64"] = fp32_error_vs_fp64(bpm, cases, Rs, kept)
    legs = {}
    want = set() if args.legs == "none" else set(args.legs.split(","))
    if "cfg0" in want:
        # the batch takes the kernel family the autotuner measures fastest for 64 solves of this size
        t64 = None if args.no_autotune else bpm.autotune("f64", 4096, 0, nsolves=64, nsteps=200)
        t32 = None if args.no_autotune else bpm.autotune("f32", 4096, 0, nsolves=64, nsteps=200)
        r64 = leg_batch(bpm, torch, synth.flat_bragg_scan(n_angles=64, precision="f64"), "cfg0 FP64", steps=3,
                        warmup=1)
        r32 = leg_batch(bpm, torch, synth.flat_bragg_scan(n_angles=64, precision="f32"), "cfg0 FP32", steps=3,
                        warmup=1, keep=(0, 31, 63))
        legs["cfg0_angle_scan"] = {
            "workload": "64-angle scan across the Darwin width, flat symmetric Bragg slab, Nx 4096, Nz 2000, "
                        "one batch launch",
            "f64_value": r64["value"], "f64_ms": r64["ms_per_step"],
            "f32_value": r32["value"], "f32_ms": r32["ms_per_step"], "unit": "cell-steps/s",
            "f32_error_vs_fp64": r32["fp32_error_vs_fp64"],
            "autotune": {"f64": t64, "f32": t32}}
        for prec in ("f64", "f32"):
            bpm.schedule_set(prec, 4096, 0, "default")
    if "cfg0x4" in want:
        # config 0's scan replicated four times (256 solves, one per compute unit):
        # the GPU-filling run for config 0's roofline
        rep = {}
        for pr in ("f64", "f32"):
            scan = synth.flat_bragg_scan(n_angles=64, precision=pr)
            cases4 = [(dict(p), psi) for _ in range(4) for p, psi in scan]
            r = leg_batch(bpm, torch, cases4, "cfg0 x4 %s" % pr, steps=3, warmup=1)
            rep[pr] = {"value": r["value"], "ms": r["ms_per_step"], "roofline": alu_roofline(cases4, r["ms_per_step"], pr)}
        legs["cfg0_replicated_x4"] = dict(
            rep, unit="cell-steps/s",
            workload="config 0's 64-angle scan replicated 4 times: 256 solves of Nx 4096 x Nz 2000 in one batch "
                     "launch (per-size kernel), labelled as a replica so the batch fills the 256 compute units")
    if "cfg1f64" in want and cfg["workload"] == "bent_laue" and prec == "f32":
        # the headline workload marched in FP64: FP32 against FP64 at equal batching
        c64 = [(dict(p, precision="f64"), psi) for p, psi in cases]
        r = leg_batch(bpm, torch, c64, "cfg1 FP64", steps=2, warmup=1)
        legs["cfg1_fp64_batch"] = {
            "workload": "the headline batch (255 bent-Laue solves, Nx 16384 x Nz 8000) in FP64, one launch",
            "value": r["value"], "ms_per_step": r["ms_per_step"], "unit": "cell-steps/s",
            "roofline": alu_roofline(c64, r["ms_per_step"], "f64"),
            "fp32_over_fp64_equal_batching": value / r["value"]}
    if "cfg2" in want:
        legs["cfg2_dislocation"] = dict(
            leg_batch(bpm, torch, synth.disl_bragg_cores(256), "cfg2", keep=(137,)),
            workload="asymmetric Bragg trapezoid + edge dislocation, Nx 32768, Nz 16000, FP32, "
                     "256 seeded core positions")
    if "cfg3" in want:
        legs["cfg3_td_batch"] = dict(
            leg_batch(bpm, torch, synth.td_batch(), "cfg3", keep=(0, 511, 1023)),
            workload="1024 spectral components of a 20 fs pulse, Nx 2048-16384, Nz 1000-8000, FP32, "
                     "one mixed-size launch")
    if "next" in want:
        legs["next_rows"] = leg_next(bpm, torch, synth)
    if "3d" in want:
        cube = [synth.cube_3d(seed=synth.SEED_BASE + 5 + k) for k in range(256)]
        print("leg 3d single (wide lane)", file=sys.stderr, flush=True)
        wide = time_single(bpm, torch, cube[0], steps=3, warmup=1)
        one = leg_batch(bpm, torch, cube[:1], "3d single, one workgroup", steps=1, warmup=1)
        many = leg_batch(bpm, torch, cube, "3d batch", steps=1, warmup=1, keep=(0,))
        legs["paper_3d"] = {
            "workload": "3D envelopes 512 x 256 x 300 steps (the paper's 300 x 200 x 300 3D case padded to "
                        "powers of two), 10 um cube with an edge dislocation, FP32",
            "single_solve_ms": wide["ms"], "single_value": wide["value"],
            "single_one_workgroup_ms": one["ms_per_step"],
            "batch_solves": many["solves"], "value": many["value"], "unit": "cell-steps/s",
            "fp32_error_vs_fp64": many["fp32_error_vs_fp64"],
            "paper_context": "about 13 s per realization on a Perlmutter node (Python package; CPU or GPU not stated)"}
        print("leg single large solves (wide lane)", file=sys.stderr, flush=True)
        big = {}
        for prec in ("f32", "f64"):
            case = synth.flat_bragg_scan(n_angles=1, nx=65536, nz=2000, precision=prec)[0]
            big[prec] = time_single(bpm, torch, case, steps=2, warmup=1)
        legs["single_large"] = {
            "workload": "one flat-Bragg solve Nx 65536 x Nz 2000 alone through bpm_propagate_device (wide lane)",
            "f32_ms": big["f32"]["ms"], "f32_value": big["f32"]["value"],
            "f64_ms": big["f64"]["ms"], "f64_value": big["f64"]["value"], "unit": "cell-steps/s"}
    if "cfg4" in want:
        legs["cfg4_serving"] = dict(
            leg_serve(bpm, synth, args.serve_requests, args.serve_rate, args.serve_budget_gb, args.serve_chunk),
            workload="Poisson stream, Nx 1024-65536 log-uniform, Nz 500-20000, flat/bent/dislocation/"
                     "trapezoid, 20% FP64")
    if legs:
        out["legs"] = legs
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cases)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
