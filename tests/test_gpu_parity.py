"""Parity of the HIP march (through the C ABI) with the FP64 oracle.

Bars (tests/bars.py): FP64 path relative L2 <= 1e-10 on the exit envelopes,
FP32 path <= 1e-4; FP32 |dR|, |dT| <= 1e-5; FP64 |dR|, |dT| within the bound
the envelope bar implies, 2 tol sqrt(X) + tol^2.  Relative L2 is taken over the
pair (psi+, psi-) of a solve.  Inputs are seeded and identical on both sides.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from bars import TOL, r_bar, t_bar
from paper_2601_06340_amd import synth

pytestmark = pytest.mark.gpu

# R and T of the same envelopes summed in two groupings (per thread vs per
# workgroup): FP64 sums of n <= 2^18 non-negative terms, whose rounding-order
# differences are of order sqrt(n) 2^-53 ~ 6e-14
SUM_ORDER_RTOL = 1e-13


def bpm():
    from paper_2601_06340_amd import bpm as b
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return b


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_pair(gp, gm, op, om):
    g = np.concatenate([np.ravel(gp), np.ravel(gm)])
    o = np.concatenate([np.ravel(op), np.ravel(om)])
    return float(np.linalg.norm(g - o) / np.linalg.norm(o))


def check(p, psi_p0, psi_m0=None, label=""):
    B = bpm()
    prec = p["precision"]
    say("case", label, "nx", p["nx"], "nz", p["nz"], prec)
    plan = B.Plan(p)
    gp, gm, gR, gT = plan.propagate(psi_p0, psi_m0)
    op, om, oR, oT = oracle.propagate(p, psi_p0, psi_m0)
    err = rel_pair(gp, gm, op, om)
    tol = TOL[prec][0]
    say("   rel L2 %.3e  dR %.2e  dT %.2e" % (err, abs(gR - oR), abs(gT - oT)))
    assert err <= tol, (label, err)
    assert abs(gR - oR) <= r_bar(prec, oR) and abs(gT - oT) <= t_bar(prec, oT), (label, gR, oR, gT, oT)
    plan.close()
    return err


def with_prec(p, prec):
    q = dict(p)
    q["precision"] = prec
    return q


# ------------------------------------------------------------------ every kernel size
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("log2n", list(range(6, 17)))
def test_every_uniform_size_random_fields_ragged_mask(prec, log2n):
    B = bpm()
    nx = 1 << log2n
    if nx > B.max_nx(prec):
        pytest.skip("beyond this precision's resident lane")
    nz = 40
    # ragged mask: interval edges off every tile boundary, changing per step
    seg = np.zeros((nz, 1, 2), np.int32)
    for n in range(nz):
        seg[n, 0] = (min(nx, 3 + 7 * n % (nx // 3)), max(0, nx - 5 - 11 * n % (nx // 4)))
    p = synth.base_problem(nx, nz, 0.1, 0.05, seg, precision=prec, det=(nx // 7, nx - nx // 5))
    a, b = synth.random_envelopes(nx, 100 + log2n)
    check(p, a, 0.3 * b, "uniform-%d" % nx)


def test_shared_propagator_table_outlives_its_first_plan():
    """Plans of the same geometry share one propagator table: destroying the
    plan that built it leaves the others correct, and a plan that differs only
    in dz gets a table of its own."""
    B = bpm()
    nx, nz = 1024, 60
    seg = np.tile(np.array([[[100, 900]]], np.int32), (nz, 1, 1))
    a, _ = synth.random_envelopes(nx, 7)
    p1 = synth.base_problem(nx, nz, 0.1, 0.05, seg, precision="f64")
    p2 = dict(p1, chih=complex(-1.2e-6, 5e-9), chihb=complex(-1.2e-6, 5e-9))
    p3 = dict(p1, dz_um=0.04)
    first = B.Plan(p1)
    second = B.Plan(p2)
    third = B.Plan(p3)
    first.close()
    for plan, p, label in ((second, p2, "shared"), (third, p3, "own")):
        gp, gm, _, _ = plan.propagate(a, None)
        op, om, _, _ = oracle.propagate(p, a, None)
        err = rel_pair(gp, gm, op, om)
        say("   %s table: rel L2 %.3e" % (label, err))
        assert err <= TOL["f64"][0]
        plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_far_field_equals_one_vacuum_step(prec):
    """bpm_far_field: exit envelopes of a crystal solve carried 2 m and 4 m through
    vacuum, against the oracle's single vacuum step of that length."""
    B = bpm()
    p, psi = synth.flat_bragg_scan(n_angles=1, nx=4096, nz=200, precision=prec)[0]
    plan = B.Plan(p)
    ep, em, _, _ = plan.propagate(psi)
    tol = TOL[prec][0]
    for D in (2.0e6, 4.0e6, 2.0e6):
        fp, fm = plan.far_field(D, ep, em)
        v = dict(p, nz=1, dz_um=D, seg=synth.mask_empty(1), strain={"kind": "none"})
        op, om, _, _ = oracle.propagate(v, ep, em)
        err = rel_pair(fp, fm, op, om)
        say("   far field %.0e um rel L2 %.3e" % (D, err))
        assert err <= tol
    with pytest.raises(B.BpmError) as e:
        plan.far_field(-1.0, ep, em)
    assert e.value.status == B.E_INVALID
    plan.close()


# ------------------------------------------------------------------ physics workloads
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_flat_bragg_scan_small(prec):
    cases = synth.flat_bragg_scan(n_angles=4, nx=2048, nz=600, precision=prec)
    for i, (p, psi) in enumerate(cases):
        check(p, psi, label="bragg-%d" % i)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_bent_laue_small(prec):
    cases = synth.bent_laue(radii_m=(1.0, 0.1), nx=2048, nz=800, thickness=20.0, precision=prec)
    for i, (p, psi) in enumerate(cases):
        check(p, psi, label="bent-%d" % i)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_dislocation_trapezoid_small(prec):
    p, psi = synth.disl_bragg(nx=4096, nz=1000, scale=0.125, precision=prec)
    check(p, psi, label="disl")


@pytest.mark.parametrize("prec,nx", [("f64", 4096), ("f32", 4096), ("f32", 32768)])
def test_dislocation_with_fractional_burgers_vector(prec, nx):
    """b/d not a whole number (the library's general arctangent path; whole
    numbers take the algebraic winding path, covered above)."""
    p, psi = synth.disl_bragg(nx=nx, nz=200, scale=nx / 32768 * 0.125 if nx > 4096 else 0.125, precision=prec)
    p["strain"] = dict(p["strain"], b_um=0.3e-3)
    check(p, psi, label="disl-frac-b-%d" % nx)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_strain_table_and_two_interval_mask(prec):
    nx, nz = 1024, 300
    dx, dz = 0.1, 0.05
    verts = [(10.0, 2.0), (80.0, 2.0), (80.0, 14.0), (60.0, 14.0), (60.0, 6.0), (30.0, 6.0),
             (30.0, 14.0), (10.0, 14.0)]  # a U: two intervals per step above z = 6
    seg = synth.mask_polygon(nz, nx, dx, dz, verts, nseg=2)
    assert (seg[:, 1, 1] > seg[:, 1, 0]).any(), "polygon should need two intervals somewhere"
    rng = synth.SplitMix64(77)
    u = np.array([[1e-4 * math.sin(0.01 * j + 0.02 * n) + 2e-6 * rng.uniform() for j in range(nx)]
                  for n in range(nz)])
    p = synth.base_problem(nx, nz, dx, dz, seg, precision=prec,
                           strain={"kind": "table", "u_table": u})
    psi = synth.gaussian_beam(nx, dx, 30.0, 8.0, synth.envelope_tilt(synth.LAMBDA_UM, synth.D_UM, 2e-6))
    check(p, psi, label="table-polygon")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_zero_steps_and_empty_crystal(prec):
    nx = 512
    a, b = synth.random_envelopes(nx, 9)
    p0 = synth.base_problem(nx, 0, 0.1, 0.05, synth.mask_empty(0), precision=prec, det=(10, 300))
    check(p0, a, b, "nz=0")
    p1 = synth.base_problem(nx, 50, 0.1, 0.05, synth.mask_empty(50), precision=prec)
    check(p1, a, b, "vacuum")


# ------------------------------------------------------------------ staged (four-step) sizes
@pytest.mark.parametrize("prec,nx", [("f32", 32768), ("f64", 16384), ("f64", 32768)])
def test_staged_bent_laue(prec, nx):
    cases = synth.bent_laue(radii_m=(0.5,), nx=nx, nz=240, thickness=6.0, precision=prec)
    p, psi = cases[0]
    check(p, psi, label="staged-bent-%d" % nx)


@pytest.mark.parametrize("prec,nx", [("f32", 32768), ("f64", 16384)])
def test_staged_dislocation_trapezoid(prec, nx):
    p, psi = synth.disl_bragg(nx=nx, nz=300, scale=nx / 32768 * 0.04, precision=prec)
    check(p, psi, label="staged-disl-%d" % nx)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_staged_strain_table_ragged_two_intervals(prec):
    nx = 16384 if prec == "f64" else 32768
    nz = 60
    seg = np.zeros((nz, 2, 2), np.int32)
    for n in range(nz):
        seg[n, 0] = (17 + 13 * n, nx // 3 + 5 * n)
        seg[n, 1] = (nx // 2 - 7 * n, nx - 19 - 3 * n)
    rng = synth.SplitMix64(91)
    u = np.array([[2e-4 * math.sin(0.003 * j + 0.05 * n) + 1e-6 * rng.uniform() for j in range(nx)]
                  for n in range(nz)])
    p = synth.base_problem(nx, nz, 0.1, 0.05, seg, precision=prec, det=(nx // 9, nx - nx // 7),
                           strain={"kind": "table", "u_table": u})
    a, b = synth.random_envelopes(nx, 5)
    check(p, a, 0.5 * b, "staged-table")


# ------------------------------------------------------------------ higher-order splittings (Eq. (13))
@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("prec,nx", [("f64", 1024), ("f32", 1024), ("f64", 8192), ("f32", 16384),
                                     ("f64", 16384), ("f32", 32768)])
def test_split_order_bent_laue(order, prec, nx):
    """z-dependent strain: every coupling sub-step samples its own height."""
    p, psi = synth.bent_laue(radii_m=(0.3,), nx=nx, nz=60, thickness=2.0, precision=prec)[0]
    p["split_order"] = order
    check(p, psi, label="split%d-bent-%d" % (order, nx))


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_split_order_masks_dislocation_and_table(order, prec):
    p, psi = synth.flat_bragg_scan(n_angles=1, nx=2048, nz=120, precision=prec)[0]
    p["split_order"] = order
    check(p, psi, label="split%d-bragg" % order)
    p, psi = synth.disl_bragg(nx=4096, nz=150, scale=0.125, precision=prec)
    p["split_order"] = order
    check(p, psi, label="split%d-disl" % order)
    nx, nz = 512, 80
    rng = synth.SplitMix64(5)
    u = np.array([[3e-5 * math.sin(0.02 * j + 0.1 * n) + 1e-6 * rng.uniform() for j in range(nx)]
                  for n in range(nz)])
    seg = np.zeros((nz, 2, 2), np.int32)
    for n in range(nz):
        seg[n, 0] = (20 + n, 200)
        seg[n, 1] = (260, 500 - n)
    p = synth.base_problem(nx, nz, 0.1, 0.05, seg, precision=prec, strain={"kind": "table", "u_table": u})
    p["split_order"] = order
    a, b = synth.random_envelopes(nx, 3)
    check(p, a, 0.2 * b, "split%d-table" % order)


def test_split_orders_mixed_in_one_batch_and_chunked_server():
    B = bpm()
    import torch
    cases = []
    for k, (order, nx) in enumerate(((1, 2048), (2, 4096), (4, 1024), (2, 32768), (4, 16384))):
        p, psi = synth.bent_laue(radii_m=(0.5 + k,), nx=nx, nz=40 + 7 * k, thickness=1.5, precision="f32")[0]
        p["split_order"] = order
        cases.append((p, psi))
    plans = [B.Plan(p) for p, _ in cases]
    batch = B.Batch(plans)
    buf = batch.pack([(psi, None) for _, psi in cases])
    rt = torch.zeros(2 * len(plans), dtype=torch.float64, device="cuda")
    batch.run(buf.data_ptr(), buf.data_ptr(), rt.data_ptr())
    torch.cuda.synchronize()
    outs = batch.unpack(buf)
    for i, (p, psi) in enumerate(cases):
        op, om, oR, _ = oracle.propagate(p, psi)
        err = rel_pair(outs[i][0], outs[i][1], op, om)
        say("split batch", i, p["split_order"], p["nx"], "%.3e" % err)
        assert err <= TOL["f32"][0]
        assert abs(rt.cpu().numpy()[2 * i] - oR) <= r_bar("f32", oR)
    srv = B.Server(hbm_budget_bytes=1 << 30, max_slots=8, chunk_steps=5)
    ts = [srv.submit(p, psi) for p, psi in cases]
    assert srv.drain(120.0)
    for t, (p, psi) in zip(ts, cases):
        r = srv.poll(t)
        assert r["status"] == 0
        op, om, _, _ = oracle.propagate(p, psi)
        assert rel_pair(r["psi_p"], r["psi_m"], op, om) <= TOL["f32"][0]
    srv.close()


def test_fp32_long_march_error_budget():
    """Nz = 8000 FP32 Bragg solve stays inside the FP32 bars (no linear drift)."""
    cases = synth.flat_bragg_scan(n_angles=1, nx=4096, nz=8000, precision="f32")
    p, psi = cases[0]
    err = check(p, psi, label="fp32-8000")
    assert err <= 5e-5


@pytest.mark.parametrize("nx,tilt", [(8192, 0.0), (2048, 0.0), (16384, 0.0), (8192, 0.3)])
def test_fp32_vacuum_march_keeps_power(nx, tilt):
    """A wide beam that never meets the crystal, 4000 FP32 steps of pure
    propagation: T stays 1 within the FP32 bar and the envelopes match the
    oracle.  Its energy sits in a few low-frequency bins that turn by less than
    2e-4 rad per step, where the -theta^2/2 that keeps |P| = 1 lies below half
    an ulp: adding it to the propagated value on its own drops it at every step
    (T grew by 8e-5 over these 4000 steps)."""
    dx, dz, nz = 0.1, 0.05, 4000
    Lx = nx * dx
    seg = synth.mask_x_slab(nz, nx, dx, 0.9 * Lx, 0.95 * Lx)
    p = synth.base_problem(nx, nz, dx, dz, seg, det=(0, nx), precision="f32")
    psi = synth.gaussian_beam(nx, dx, 0.3125 * Lx, 50.0, tilt)
    check(p, psi, label="vacuum nx %d tilt %g" % (nx, tilt))


@pytest.mark.parametrize("nz", [2000, 8000, 16000])
def test_fp32_gate_lengths_every_kernel_family(nz):
    """The FP32 bars at Nz = 2000, 8000 and 16000 (config 0's crystal, Nx 4096,
    three angles across the Darwin width), through the per-size kernel (single
    plans) and through batches on the mixed-size and any-size kernels."""
    B = bpm()
    import torch
    cases = synth.flat_bragg_scan(n_angles=3, nx=4096, nz=nz, precision="f32")
    ores, oR, oT = oracle.propagate_batch([p for p, _ in cases], [(psi, None) for _, psi in cases])
    tol = TOL["f32"][0]
    for i, (p, psi) in enumerate(cases):
        pl = B.Plan(p)
        gp, gm, gR, gT = pl.propagate(psi)
        pl.close()
        err = rel_pair(gp, gm, ores[i][0], ores[i][1])
        say("gate nz %d single %d rel L2 %.3e dR %.2e dT %.2e" % (nz, i, err, abs(gR - oR[i]), abs(gT - oT[i])))
        assert err <= tol and abs(gR - oR[i]) <= r_bar("f32", oR[i]) and abs(gT - oT[i]) <= t_bar("f32", oT[i])
    for sched in ("mixed", "any"):
        B.schedule_set("f32", 4096, 0, sched)
        try:
            plans = [B.Plan(p) for p, _ in cases]
            batch = B.Batch(plans)
            buf = batch.pack([(psi, None) for _, psi in cases])
            rt = torch.zeros(2 * len(plans), dtype=torch.float64, device="cuda")
            batch.run(buf.data_ptr(), buf.data_ptr(), rt.data_ptr())
            torch.cuda.synchronize()
            outs = batch.unpack(buf)
            batch.close()
            for pl in plans:
                pl.close()
        finally:
            B.schedule_set("f32", 4096, 0, "default")
        rt = rt.cpu().numpy()
        for i in range(len(cases)):
            err = rel_pair(outs[i][0], outs[i][1], ores[i][0], ores[i][1])
            say("gate nz %d %s %d rel L2 %.3e dR %.2e" % (nz, sched, i, err, abs(rt[2 * i] - oR[i])))
            assert err <= tol and abs(rt[2 * i] - oR[i]) <= r_bar("f32", oR[i]) and abs(rt[2 * i + 1] - oT[i]) <= t_bar("f32", oT[i])


# ------------------------------------------------------------------ batches
def test_uniform_batch_bitwise_equals_single_solves():
    B = bpm()
    import torch
    cases = synth.flat_bragg_scan(n_angles=5, nx=1024, nz=300, precision="f32")
    plans = [B.Plan(p) for p, _ in cases]
    batch = B.Batch(plans)
    buf = batch.pack([(psi, None) for _, psi in cases])
    rt = torch.zeros(2 * len(plans), dtype=torch.float64, device="cuda")
    batch.run(buf.data_ptr(), buf.data_ptr(), rt.data_ptr())
    torch.cuda.synchronize()
    outs = batch.unpack(buf)
    rt = rt.cpu().numpy()
    for i, (pl, (p, psi)) in enumerate(zip(plans, cases)):
        sp, sm, sR, sT = pl.propagate(psi)
        assert np.array_equal(outs[i][0], sp) and np.array_equal(outs[i][1], sm)
        assert rt[2 * i] == sR and rt[2 * i + 1] == sT


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_mixed_size_batch_one_launch_matches_oracle(prec):
    B = bpm()
    import torch
    cases = synth.td_batch(n_comp=6, nx_choices=(1024, 2048, 4096, 8192), nz_range=(200, 500),
                           precision=prec)
    plans = [B.Plan(p) for p, _ in cases]
    batch = B.Batch(plans)
    buf = batch.pack([(psi, None) for _, psi in cases])
    rt = torch.zeros(2 * len(plans), dtype=torch.float64, device="cuda")
    batch.run(buf.data_ptr(), buf.data_ptr(), rt.data_ptr())
    torch.cuda.synchronize()
    outs = batch.unpack(buf)
    rt = rt.cpu().numpy()
    ores, oR, oT = oracle.propagate_batch([p for p, _ in cases], [(psi, None) for _, psi in cases])
    tol = TOL[prec][0]
    for i in range(len(cases)):
        err = rel_pair(outs[i][0], outs[i][1], ores[i][0], ores[i][1])
        say("mixed", i, cases[i][0]["nx"], cases[i][0]["nz"], "%.3e" % err)
        assert err <= tol
        assert abs(rt[2 * i] - oR[i]) <= r_bar(prec, oR[i]) and abs(rt[2 * i + 1] - oT[i]) <= t_bar(prec, oT[i])


def test_staged_sizes_in_batch_and_chunked_server_equal_single_solves():
    """A batch holding staged and register-resident sizes reproduces the single
    solves bitwise, and so does a staged solve marched in server chunks (its
    state returns to natural order between launches)."""
    B = bpm()
    import torch
    cases = [synth.bent_laue(radii_m=(0.7,), nx=32768, nz=150, thickness=4.0, precision="f32")[0],
             synth.flat_bragg_scan(n_angles=1, nx=4096, nz=150, precision="f32")[0],
             synth.bent_laue(radii_m=(2.0,), nx=65536, nz=90, thickness=3.0, precision="f32")[0]]
    plans = [B.Plan(p) for p, _ in cases]
    batch = B.Batch(plans)
    buf = batch.pack([(psi, None) for _, psi in cases])
    rt = torch.zeros(2 * len(plans), dtype=torch.float64, device="cuda")
    batch.run(buf.data_ptr(), buf.data_ptr(), rt.data_ptr())
    torch.cuda.synchronize()
    outs = batch.unpack(buf)
    rt = rt.cpu().numpy()
    singles = []
    for i, (pl, (p, psi)) in enumerate(zip(plans, cases)):
        sp, sm, sR, sT = pl.propagate(psi)
        singles.append((sp, sm, sR))
        say("staged batch", i, p["nx"], "bitwise", np.array_equal(outs[i][0], sp))
        assert np.array_equal(outs[i][0], sp) and np.array_equal(outs[i][1], sm)
        # a staged size marched alone runs in the wide lane: R, T summed per workgroup
        assert abs(rt[2 * i] - sR) <= SUM_ORDER_RTOL * abs(sR) and abs(rt[2 * i + 1] - sT) <= SUM_ORDER_RTOL * abs(sT)
    op, om, oR, _ = oracle.propagate(*cases[2])
    assert rel_pair(singles[2][0], singles[2][1], op, om) <= TOL["f32"][0]
    srv = B.Server(hbm_budget_bytes=1 << 30, max_slots=8, chunk_steps=37)
    t = srv.submit(*cases[0])
    assert srv.drain(120.0)
    r = srv.poll(t)
    assert r["status"] == 0
    assert np.array_equal(r["psi_p"], singles[0][0]) and np.array_equal(r["psi_m"], singles[0][1])
    # the server marches staged sizes in the any-size kernel, a single solve
    # alone runs in the wide lane: same envelopes, FP64 power sums grouped
    # differently
    assert abs(r["R"] - singles[0][2]) <= SUM_ORDER_RTOL * abs(singles[0][2])
    srv.close()


# ------------------------------------------------------------------ wide lane
def _wide_case(name):
    """Staged-size and 3D solves for the wide lane: graph blocks of 32 steps plus
    remainders, every splitting order (order 2 starts with a leading coupling)."""
    disl = {"kind": "edge_dislocation", "x_ref_um": 25.5, "z_ref_um": 1.2, "b_um": 4 * synth.D_UM, "nu": 0.22}
    if name == "f32-32768-bent":
        p, psi = synth.bent_laue(radii_m=(0.7,), nx=32768, nz=70, thickness=4.0, precision="f32")[0]
        return p, psi, None
    if name == "f64-16384-bragg-o2":
        p, psi = synth.flat_bragg_scan(n_angles=1, nx=16384, nz=40, precision="f64")[0]
        p["split_order"] = 2
        return p, psi, None
    if name == "f32-65536-disl-o4":
        p, psi = synth.disl_bragg(nx=65536, nz=33, scale=0.125, precision="f32")
        p["split_order"] = 4
        return p, psi, None
    if name == "f64-65536-bent-short":
        p, psi = synth.bent_laue(radii_m=(2.0,), nx=65536, nz=20, thickness=1.0, precision="f64")[0]
        return p, psi, None
    if name == "3d-f32-256-disl":
        p, a, b = _problem3d(256, 40, "f32", strain=disl)
        return p, a, b
    if name == "3d-f64-16-o2":
        p, a, b = _problem3d(16, 35, "f64", order=2)
        return p, a, b
    if name == "3d-f64-1024x16-disl-o2":
        d2 = dict(disl, x_ref_um=51.25)
        p, a, b = _problem3d(16, 35, "f64", strain=d2, order=2, nx=1024)
        return p, a, b
    if name == "3d-f32-256x128":
        p, a, b = _problem3d(128, 40, "f32", nx=256)
        return p, a, b
    raise KeyError(name)


WIDE_CASES = ["f32-32768-bent", "f64-16384-bragg-o2", "f32-65536-disl-o4", "f64-65536-bent-short",
              "3d-f32-256-disl", "3d-f64-16-o2", "3d-f64-1024x16-disl-o2", "3d-f32-256x128"]


@pytest.mark.parametrize("name", WIDE_CASES)
def test_wide_lane_matches_one_workgroup_march_and_oracle(name):
    """A staged-size or 3D solve marched alone spreads over the device (row and
    column launches, graphs of 32 steps): its envelopes equal the one-workgroup
    march's bitwise on every call (three calls on fresh buffers with other
    device work in between replay the recorded graph), and R, T agree to a few
    ulps (partial sums per workgroup instead of per thread)."""
    B = bpm()
    import torch
    p, a, b = _wide_case(name)
    say("wide", name, "nx", p["nx"], "ny", p.get("ny", 1), "nz", p["nz"], p["precision"])
    plan = B.Plan(p)
    one = B.Batch([plan])
    buf = one.pack([(a, b)])
    rt1 = torch.zeros(2, dtype=torch.float64, device="cuda")
    one.run(buf.data_ptr(), buf.data_ptr(), rt1.data_ptr())
    torch.cuda.synchronize()
    ref = one.unpack(buf)[0]
    rt1 = rt1.cpu().numpy()
    for rep in range(3):
        src = one.pack([(a, b)])
        dst = torch.empty_like(src)
        rt = torch.zeros(2, dtype=torch.float64, device="cuda")
        plan.propagate_device(src.data_ptr(), dst.data_ptr(), rt.data_ptr())
        junk = torch.randn(1 << 20, device="cuda").sum()   # unrelated device work between replays
        torch.cuda.synchronize()
        got = one.unpack(dst)[0]
        rt = rt.cpu().numpy()
        say("   call", rep, "bitwise", np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]),
            "R %.17g vs %.17g" % (rt[0], rt1[0]), float(junk) * 0)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        assert abs(rt[0] - rt1[0]) <= SUM_ORDER_RTOL * abs(rt1[0])
        assert abs(rt[1] - rt1[1]) <= SUM_ORDER_RTOL * abs(rt1[1])
    op, om, oR, oT = oracle.propagate(p, a, b)
    err = rel_pair(got[0], got[1], op, om)
    tol = TOL[p["precision"]][0]
    say("   oracle rel L2 %.3e  dR %.2e" % (err, abs(rt[0] - oR)))
    assert err <= tol and abs(rt[0] - oR) <= r_bar(p["precision"], oR) and abs(rt[1] - oT) <= t_bar(p["precision"], oT)
    one.close()
    plan.close()


@pytest.mark.parametrize("nz", [0, 1])
@pytest.mark.parametrize("name", ["f32-32768-bent", "3d-f64-16-o2"])
def test_wide_lane_degenerate_marches(name, nz):
    """nz = 0 (entry and detector sums only: the output is the input, R and T
    its powers) and nz = 1 (one step, no graph) in the wide lane, against the
    oracle and the one-workgroup march."""
    B = bpm()
    import torch
    p, a, b = _wide_case(name)
    p = dict(p, nz=nz)
    p["seg"] = np.asarray(p["seg"])[:nz]
    plan = B.Plan(p)
    one = B.Batch([plan])
    buf = one.pack([(a, b)])
    dst = torch.empty_like(buf)
    rt = torch.zeros(2, dtype=torch.float64, device="cuda")
    plan.propagate_device(buf.data_ptr(), dst.data_ptr(), rt.data_ptr())
    rt1 = torch.zeros(2, dtype=torch.float64, device="cuda")
    one.run(buf.data_ptr(), buf.data_ptr(), rt1.data_ptr())
    torch.cuda.synchronize()
    got, ref = one.unpack(dst)[0], one.unpack(buf)[0]
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    rt, rt1 = rt.cpu().numpy(), rt1.cpu().numpy()
    op, om, oR, oT = oracle.propagate(p, a, b)
    err = rel_pair(got[0], got[1], op, om)
    say("wide nz", nz, name, "rel L2 %.3e R %.6g oracle %.6g" % (err, rt[0], oR))
    assert err <= TOL[p["precision"]][0]
    assert abs(rt[0] - oR) <= r_bar(p["precision"], oR) and abs(rt[1] - oT) <= t_bar(p["precision"], oT)
    assert abs(rt[0] - rt1[0]) <= SUM_ORDER_RTOL * abs(rt1[0]) and abs(rt[1] - rt1[1]) <= SUM_ORDER_RTOL * abs(rt1[1])
    one.close()
    plan.close()


def test_server_marches_long_3d_request_in_the_wide_lane():
    """A long 3D request (estimated one-workgroup march > 0.5 s) runs wide in the
    server and equals the single-solve march bitwise."""
    B = bpm()
    p, a, b = _problem3d(256, 2000, "f32", seed=3)   # estimated one-workgroup march 0.52 s
    plan = B.Plan(p)
    rp, rm, rR, rT = plan.propagate(a, b)
    plan.close()
    srv = B.Server(hbm_budget_bytes=4 << 30, max_slots=4, chunk_steps=100)
    t = srv.submit(p, a, b)
    assert srv.drain(120.0)
    st = srv.stats()
    assert st["wide"] == 1
    r = srv.poll(t)
    assert r["status"] == 0
    assert np.array_equal(r["psi_p"], rp) and np.array_equal(r["psi_m"], rm)
    assert abs(r["R"] - rR) <= SUM_ORDER_RTOL * abs(rR) and abs(r["T"] - rT) <= SUM_ORDER_RTOL * abs(rT)
    srv.close()


def test_server_marches_long_staged_solves_in_the_wide_lane():
    """A long staged-size request (estimated one-workgroup march > 0.5 s) runs in
    the server's wide lane in chunks of 2*chunk_steps z-steps (graph blocks and
    remainders, natural order between chunks): its envelopes equal the
    single-solve march's bitwise; the regular requests beside it still match the
    oracle."""
    B = bpm()
    long_p, long_psi = synth.flat_bragg_scan(n_angles=1, nx=65536, nz=4000, precision="f32")[0]
    small = [synth.flat_bragg_scan(n_angles=1, nx=2048, nz=300, precision="f32")[0],
             synth.bent_laue(radii_m=(1.0,), nx=8192, nz=200, thickness=1.0, precision="f64")[0]]
    plan = B.Plan(long_p)
    rp, rm, rR, rT = plan.propagate(long_psi)
    plan.close()
    srv = B.Server(hbm_budget_bytes=4 << 30, max_slots=8, chunk_steps=300)
    t_long = srv.submit(long_p, long_psi)
    t_small = [srv.submit(p, psi) for p, psi in small]
    assert srv.drain(120.0)
    st = srv.stats()
    say("server wide solves", st["wide"], "launches", st["launches"])
    assert st["wide"] == 1 and st["completed"] == 3
    r = srv.poll(t_long)
    assert r["status"] == 0
    assert np.array_equal(r["psi_p"], rp) and np.array_equal(r["psi_m"], rm)
    assert abs(r["R"] - rR) <= SUM_ORDER_RTOL * abs(rR) and abs(r["T"] - rT) <= SUM_ORDER_RTOL * abs(rT)
    for t, (p, psi) in zip(t_small, small):
        x = srv.poll(t)
        assert x["status"] == 0
        op, om, _, _ = oracle.propagate(p, psi)
        assert rel_pair(x["psi_p"], x["psi_m"], op, om) <= TOL[p["precision"]][0]
    srv.close()


def test_server_moves_a_running_solve_to_the_wide_lane():
    """With more than 64 other solves in the first round the long request starts
    in the rounds (one workgroup, any-size kernel); once they have finished it
    moves to the wide lane part way through.  Its envelopes still equal the
    single-solve march's bitwise."""
    B = bpm()
    long_p, long_psi = synth.flat_bragg_scan(n_angles=1, nx=65536, nz=8000, precision="f32")[0]
    plan = B.Plan(long_p)
    rp, rm, rR, rT = plan.propagate(long_psi)
    plan.close()
    srv = B.Server(hbm_budget_bytes=4 << 30, max_slots=128, chunk_steps=300)
    # about 8 rounds each; admitted in arrival order, so all of them are in the
    # rounds when the long request's plan is ready
    shorts = [synth.flat_bragg_scan(n_angles=1, nx=1024, nz=40000, precision="f32")[0] for _ in range(70)]
    ts = [srv.submit(p, psi, want_fields=False) for p, psi in shorts]
    t_long = srv.submit(long_p, long_psi)
    assert srv.drain(120.0)
    st = srv.stats()
    say("server wide solves", st["wide"], "launches", st["launches"])
    assert st["wide"] == 1 and st["completed"] == 71
    assert all(srv.poll(t)["status"] == 0 for t in ts)
    r = srv.poll(t_long)
    assert r["status"] == 0
    assert np.array_equal(r["psi_p"], rp) and np.array_equal(r["psi_m"], rm)
    assert abs(r["R"] - rR) <= SUM_ORDER_RTOL * abs(rR) and abs(r["T"] - rT) <= SUM_ORDER_RTOL * abs(rT)
    srv.close()


def test_autotune_and_every_schedule_match_the_oracle():
    """The autotuner times the three kernel families on a synthetic batch and
    enters the fastest; a batch marched with each schedule matches the oracle,
    and at a staged size the any-size kernel (512 threads) gives the staged
    kernel's envelopes bitwise."""
    B = bpm()
    import torch
    r = B.autotune("f32", 4096, 0, nsolves=32, nsteps=64)
    say("autotune f32 4096:", r)
    assert r["schedule"] in ("uniform", "mixed", "any") and set(r["ms"]) == {"uniform", "mixed", "any"}
    assert B.schedule_get("f32", 4096, 0) == r["schedule"]
    try:
        p, psi = synth.flat_bragg_scan(n_angles=1, nx=4096, nz=300, precision="f32")[0]
        op, om, oR, _ = oracle.propagate(p, psi)
        for sched in ("uniform", "mixed", "any"):
            B.schedule_set("f32", 4096, 0, sched)
            plan = B.Plan(p)
            batch = B.Batch([plan])
            buf = batch.pack([(psi, None)])
            rt = torch.zeros(2, dtype=torch.float64, device="cuda")
            batch.run(buf.data_ptr(), buf.data_ptr(), rt.data_ptr())
            torch.cuda.synchronize()
            gp, gm = batch.unpack(buf)[0]
            err = rel_pair(gp, gm, op, om)
            say("   schedule", sched, "rel L2 %.3e" % err)
            assert err <= TOL["f32"][0] and abs(rt.cpu().numpy()[0] - oR) <= r_bar("f32", oR)
            batch.close()
            plan.close()
        p, psi = synth.bent_laue(radii_m=(0.7,), nx=32768, nz=60, thickness=4.0, precision="f32")[0]
        outs = {}
        for sched in ("uniform", "any"):
            B.schedule_set("f32", 32768, 1, sched)
            plan = B.Plan(p)
            batch = B.Batch([plan])
            buf = batch.pack([(psi, None)])
            batch.run(buf.data_ptr(), buf.data_ptr(), None)
            torch.cuda.synchronize()
            outs[sched] = batch.unpack(buf)[0]
            batch.close()
            plan.close()
        assert np.array_equal(outs["uniform"][0], outs["any"][0]) and np.array_equal(outs["uniform"][1], outs["any"][1])
    finally:
        B.schedule_set("f32", 4096, 0, "default")
        B.schedule_set("f32", 32768, 1, "default")


@pytest.mark.parametrize("name", ["f32-32768-bent", "3d-f64-16-o2"])
def test_one_workgroup_staged_and_3d_march_matches_oracle(name):
    """The one-workgroup staged / 3D march (what batches and the server run)
    against the oracle directly."""
    B = bpm()
    import torch
    p, a, b = _wide_case(name)
    plan = B.Plan(p)
    one = B.Batch([plan])
    buf = one.pack([(a, b)])
    rt = torch.zeros(2, dtype=torch.float64, device="cuda")
    one.run(buf.data_ptr(), buf.data_ptr(), rt.data_ptr())
    torch.cuda.synchronize()
    got = one.unpack(buf)[0]
    op, om, oR, _ = oracle.propagate(p, a, b)
    err = rel_pair(got[0], got[1], op, om)
    say("one-workgroup", name, "rel L2 %.3e" % err)
    assert err <= TOL[p["precision"]][0] and abs(rt.cpu().numpy()[0] - oR) <= r_bar(p["precision"], oR)
    one.close()
    plan.close()


# ------------------------------------------------------------------ 3D envelopes
def _problem3d(ny, nz, prec, strain=None, order=1, seed=0, nx=512):
    dx, dy, dz = 0.1, 0.2, 0.05
    f = nx / 512   # the section and the detector scale with the row length
    seg = np.zeros((nz, ny, 2, 2), np.int32)
    for n in range(nz):
        for i in range(ny):   # a ragged crystal section that changes with y and z
            seg[n, i, 0] = (int(f * (40 + (7 * i + 3 * n) % 50)), int(f * (200 + (5 * i) % 60)))
            seg[n, i, 1] = (int(f * (300 - (2 * n) % 40)), int(f * (470 - (3 * i + n) % 30)))
    p = synth.base_problem(nx, nz, dx, dz, seg, precision=prec, strain=strain, det=(int(30 * f), int(480 * f)))
    p["ny"], p["dy_um"] = ny, dy
    p["split_order"] = order
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    b = 0.3 * (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx)))
    return p, a, b


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("ny", [16, 64, 256])
def test_3d_random_fields_ragged_row_masks(prec, ny):
    p, a, b = _problem3d(ny, 30, prec, seed=ny)
    check(p, a, b, "3d-%d" % ny)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_3d_strain_kinds_and_splitting(prec):
    poly = {"kind": "poly2", "x_ref_um": 25.0, "z_ref_um": 1.0, "c": [0, 1e-5, 0, 0, 4e-5, 0]}
    p, a, b = _problem3d(32, 40, prec, strain=poly, seed=1)
    check(p, a, b, "3d-poly2")
    p, a, b = _problem3d(32, 40, prec, strain=poly, order=2, seed=2)
    check(p, a, b, "3d-poly2-split2")
    disl = {"kind": "edge_dislocation", "x_ref_um": 25.05, "z_ref_um": 1.025, "b_um": 0.38e-3, "nu": 0.22}
    p, a, b = _problem3d(32, 40, prec, strain=disl, seed=3)
    check(p, a, b, "3d-disl")
    rng = synth.SplitMix64(11)
    u = np.array([[[2e-5 * math.sin(0.01 * j + 0.3 * i + 0.1 * n) + 1e-6 * rng.uniform() for j in range(512)]
                   for i in range(16)] for n in range(20)])
    p, a, b = _problem3d(16, 20, prec, strain={"kind": "table", "u_table": u}, seed=4)
    check(p, a, b, "3d-table")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nx", [256, 1024])
@pytest.mark.parametrize("ny", [16, 64, 256])
def test_3d_other_row_lengths_random_fields(prec, nx, ny):
    """Rows of 256 and 1024 samples (4 and 16 per thread), every ny: ragged row
    masks and random fields against the oracle."""
    p, a, b = _problem3d(ny, 24, prec, seed=nx + ny, nx=nx)
    check(p, a, b, "3d-%dx%d" % (nx, ny))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nx", [256, 1024])
def test_3d_other_row_lengths_strain_and_splitting(prec, nx):
    """Polynomial strain with order-2 splitting, the dislocation with order 4
    and a strain table, at rows of 256 and 1024 samples."""
    Lx = nx * 0.1
    poly = {"kind": "poly2", "x_ref_um": Lx / 2, "z_ref_um": 0.7, "c": [0, 1e-5, 0, 0, 4e-5, 0]}
    p, a, b = _problem3d(32, 30, prec, strain=poly, order=2, seed=21, nx=nx)
    check(p, a, b, "3d-%d-poly2-o2" % nx)
    disl = {"kind": "edge_dislocation", "x_ref_um": Lx / 2 + 0.05, "z_ref_um": 0.825, "b_um": 0.38e-3, "nu": 0.22}
    p, a, b = _problem3d(16, 30, prec, strain=disl, order=4, seed=22, nx=nx)
    check(p, a, b, "3d-%d-disl-o4" % nx)
    rng = synth.SplitMix64(12 + nx)
    u = np.array([[[2e-5 * math.sin(0.01 * j + 0.3 * i + 0.1 * n) + 1e-6 * rng.uniform() for j in range(nx)]
                   for i in range(16)] for n in range(12)])
    p, a, b = _problem3d(16, 12, prec, strain={"kind": "table", "u_table": u}, seed=23, nx=nx)
    check(p, a, b, "3d-%d-table" % nx)


def test_3d_row_lengths_of_one_total_size_in_one_batch():
    """256 x 64, 512 x 32 and 1024 x 16 have the same number of samples: in one
    batch each keeps its own kernel and tables and reproduces its single solve
    bitwise, and each matches the oracle."""
    B = bpm()
    import torch
    cases = [_problem3d(64, 20, "f32", seed=31, nx=256), _problem3d(32, 20, "f32", seed=32, nx=512),
             _problem3d(16, 20, "f32", seed=33, nx=1024), _problem3d(16, 20, "f64", seed=34, nx=1024)]
    plans = [B.Plan(p) for p, _, _ in cases]
    singles = [pl.propagate(a, b) for pl, (_, a, b) in zip(plans, cases)]
    batch = B.Batch(plans)
    buf = batch.pack([(a, b) for _, a, b in cases])
    rt = torch.zeros(2 * len(cases), dtype=torch.float64, device="cuda")
    batch.run(buf.data_ptr(), buf.data_ptr(), rt.data_ptr())
    torch.cuda.synchronize()
    outs = batch.unpack(buf)
    rt = rt.cpu().numpy()
    for k, ((p, a, b), s, o) in enumerate(zip(cases, singles, outs)):
        say("   3d %d x %d %s in batch bitwise" % (p["nx"], p["ny"], p["precision"]),
            np.array_equal(o[0], s[0]) and np.array_equal(o[1], s[1]))
        assert np.array_equal(o[0], s[0]) and np.array_equal(o[1], s[1])
        # a single 3D solve marches in the wide lane: same envelopes, FP64 power
        # sums grouped per workgroup
        assert abs(rt[2 * k] - s[2]) <= SUM_ORDER_RTOL * abs(s[2])
        assert abs(rt[2 * k + 1] - s[3]) <= SUM_ORDER_RTOL * abs(s[3])
        op, om, oR, oT = oracle.propagate(p, a, b)
        assert rel_pair(o[0], o[1], op, om) <= TOL[p["precision"]][0]
    batch.close()
    for pl in plans:
        pl.close()


def test_3d_batch_with_2d_solves_and_far_field():
    """3D and 2D solves in one batch reproduce their single solves bitwise; the
    far field of a 3D exit field equals the oracle's 3D vacuum step."""
    B = bpm()
    import torch
    p3, a3, b3 = _problem3d(64, 25, "f32", seed=9)
    p2, psi2 = synth.flat_bragg_scan(n_angles=1, nx=4096, nz=25, precision="f32")[0]
    plans = [B.Plan(p3), B.Plan(p2)]
    batch = B.Batch(plans)
    buf = batch.pack([(a3, b3), (psi2, None)])
    batch.run(buf.data_ptr(), buf.data_ptr())
    torch.cuda.synchronize()
    outs = batch.unpack(buf)
    s3 = plans[0].propagate(a3, b3)
    s2 = plans[1].propagate(psi2)
    assert np.array_equal(outs[0][0], s3[0]) and np.array_equal(outs[0][1], s3[1])
    assert np.array_equal(outs[1][0], s2[0])
    fp, fm = plans[0].far_field(1.0e6, s3[0], s3[1])
    ny = p3["ny"]
    v = dict(p3, nz=1, dz_um=1.0e6, seg=np.zeros((1, ny, 1, 2), np.int32), strain={"kind": "none"})
    op, om, _, _ = oracle.propagate(v, s3[0], s3[1])
    err = rel_pair(fp.reshape(-1), fm.reshape(-1), op.reshape(-1), om.reshape(-1))
    say("   3d far field rel L2 %.3e" % err)
    assert err <= TOL["f32"][0]


# ------------------------------------------------------------------ chih != chihbar (Eq. (8)-(10))
# a+ pairs with chih (the coefficient of e^{+i h x}), a- with chihbar; with the
# two unequal, a swap of them anywhere (setup, either coupling form, a kernel)
# changes the exit fields by far more than the bars
CHIH_U, CHIHB_U = complex(-1.2e-6, 3e-8), complex(-1.7e-6, -2e-8)


@pytest.mark.parametrize("order", [1, 2, 4])
@pytest.mark.parametrize("prec,nx", [("f64", 1024), ("f32", 1024), ("f64", 8192), ("f32", 16384),
                                     ("f64", 16384), ("f32", 32768)])
def test_unequal_chih_chihbar(order, prec, nx):
    p, psi = synth.bent_laue(radii_m=(0.3,), nx=nx, nz=60, thickness=2.0, precision=prec)[0]
    p["chih"], p["chihb"] = CHIH_U, CHIHB_U
    p["split_order"] = order
    _, b = synth.random_envelopes(nx, 17)
    check(p, psi, 0.3 * b, label="chih!=chihb-o%d-%d" % (order, nx))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_unequal_chih_chihbar_3d_and_dislocation(prec):
    disl = {"kind": "edge_dislocation", "x_ref_um": 25.05, "z_ref_um": 1.025, "b_um": 0.38e-3, "nu": 0.22}
    for order in (1, 2):
        p, a, b = _problem3d(32, 30, prec, strain=disl, order=order, seed=5 + order)
        p["chih"], p["chihb"] = CHIH_U, CHIHB_U
        check(p, a, b, "3d-chih!=chihb-o%d" % order)
    p, psi = synth.disl_bragg(nx=4096, nz=150, scale=0.125, precision=prec)
    p["chih"], p["chihb"] = CHIH_U, CHIHB_U
    check(p, psi, label="disl-chih!=chihb")


# ------------------------------------------------------------------ evanescent bins
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nx", [64, 1024, 16384, 32768])
def test_evanescent_bins_decay(prec, nx):
    """dx = 5e-5 um: bins with |q +/- s| > 1 take the decaying continuation of
    the propagator, exp(-dzh sqrt(p^2 - 1)) exp(-i dzh c), in the plan setup."""
    nz, dx, dz = 6, 5e-5, 2e-5
    seg = np.zeros((nz, 1, 2), np.int32)
    for n in range(nz):
        seg[n, 0] = (nx // 8 + n, nx - nx // 5)
    p = synth.base_problem(nx, nz, dx, dz, seg, precision=prec, chih=CHIH_U, chihb=CHIHB_U)
    a, b = synth.random_envelopes(nx, 23)
    check(p, a, 0.5 * b, "evanescent-%d" % nx)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_evanescent_3d_rows_decay(prec):
    """3D envelopes with dy = 2e-5 um: 2D bins beyond (qx +/- s)^2 + qy^2 = 1
    take the decaying branch of the 2D propagator in the plan setup."""
    nx, ny, nz, dy = 512, 32, 6, 2e-5
    seg3 = np.zeros((nz, ny, 1, 2), np.int32)
    seg3[:, :, 0, 1] = nx
    p = synth.base_problem(nx, nz, 0.1, 2e-5, seg3, precision=prec, chih=CHIH_U, chihb=CHIHB_U)
    p["ny"], p["dy_um"] = ny, dy
    rng = np.random.default_rng(31)
    a = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    b = 0.4 * (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx)))
    check(p, a, b, "evanescent-3d")


# ------------------------------------------------------------------ time-domain assembly
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_td_assembly_matches_oracle(prec):
    """128 pulse components on one grid, marched in one batch, assembled in time:
    the assembly alone (on the GPU's own exit envelopes) and end to end against
    the oracle's march and assembly."""
    B = bpm()
    import torch
    cases = synth.td_batch(n_comp=128, nx_choices=(1024,), nz_range=(60, 100), precision=prec)
    plans = [B.Plan(p) for p, _ in cases]
    batch = B.Batch(plans)
    buf = batch.pack([(psi, None) for _, psi in cases])
    batch.run(buf.data_ptr(), buf.data_ptr())
    td = batch.td_assemble(buf.data_ptr())
    torch.cuda.synchronize()
    td = td.cpu().to(torch.complex128).numpy()
    exits = batch.unpack(buf)
    ref = oracle.td_assemble([p for p, _ in cases], [(a, b) for a, b in exits])
    err = float(np.linalg.norm(td - ref) / np.linalg.norm(ref))
    say("   td assembly alone rel L2 %.3e" % err)
    # the carrier phase k c L is ~3e5 rad: FP64 evaluations of it (oracle and
    # kernel) each carry ~|k c L| 2^-52 ~ 6e-11 rad
    assert err <= (1e-10 if prec == "f64" else 2e-6)
    ores, _, _ = oracle.propagate_batch([p for p, _ in cases], [(psi, None) for _, psi in cases])
    ref2 = oracle.td_assemble([p for p, _ in cases], [(a, b) for a, b in ores])
    err2 = float(np.linalg.norm(td - ref2) / np.linalg.norm(ref2))
    say("   td march + assembly rel L2 %.3e" % err2)
    assert err2 <= TOL[prec][0]


def test_td_assembly_largest_m_and_invalid_m():
    B = bpm()
    import torch
    cases = synth.td_batch(n_comp=2048, nx_choices=(64,), nz_range=(5, 9), precision="f32")
    plans = [B.Plan(p) for p, _ in cases]
    batch = B.Batch(plans)
    buf = batch.pack([(psi, None) for _, psi in cases])
    batch.run(buf.data_ptr(), buf.data_ptr())
    td = batch.td_assemble(buf.data_ptr()).cpu().to(torch.complex128).numpy()
    exits = batch.unpack(buf)
    ref = oracle.td_assemble([p for p, _ in cases], [(a, b) for a, b in exits])
    err = float(np.linalg.norm(td - ref) / np.linalg.norm(ref))
    say("   td M=2048 rel L2 %.3e" % err)
    assert err <= 2e-6
    bad = B.Batch(plans[:100])
    with pytest.raises(B.BpmError) as e:
        bad.td_assemble(buf.data_ptr())
    assert e.value.status == B.E_INVALID


# ------------------------------------------------------------------ server
def test_server_alone_equals_in_mix_and_matches_oracle():
    B = bpm()
    target_p, target_psi = synth.flat_bragg_scan(n_angles=1, nx=2048, nz=700, precision="f32")[0]
    srv = B.Server(hbm_budget_bytes=1 << 30, max_slots=64, chunk_steps=128)
    t = srv.submit(target_p, target_psi)
    assert srv.drain(120.0)
    alone = srv.poll(t)
    assert alone["status"] == 0
    # now the same request in a mix of others arriving while it runs
    others = synth.td_batch(n_comp=5, nx_choices=(1024, 4096), nz_range=(300, 900), precision="f32")
    tick = [srv.submit(p, psi) for p, psi in others[:2]]
    t2 = srv.submit(target_p, target_psi)
    tick += [srv.submit(p, psi) for p, psi in others[2:]]
    assert srv.drain(120.0)
    mixed = srv.poll(t2)
    assert mixed["status"] == 0
    assert np.array_equal(alone["psi_p"], mixed["psi_p"]) and np.array_equal(alone["psi_m"], mixed["psi_m"])
    assert alone["R"] == mixed["R"]
    op, om, oR, oT = oracle.propagate(target_p, target_psi)
    assert rel_pair(mixed["psi_p"], mixed["psi_m"], op, om) <= 1e-4
    assert abs(mixed["R"] - oR) <= 1e-5
    for tk, (p, psi) in zip(tick, others):
        r = srv.poll(tk)
        assert r["status"] == 0
        op, om, oR, _ = oracle.propagate(p, psi)
        assert rel_pair(r["psi_p"], r["psi_m"], op, om) <= 1e-4
    st = srv.stats()
    assert st["completed"] == 7 and st["failed"] == 0
    srv.close()


def test_server_more_solves_than_compute_units():
    """400 long requests at once, more than there are compute units (the
    any-size launch then runs in layers of workgroups): every request
    completes, copies of one request give bitwise the same result wherever
    they sat in the launches, and a sample matches the oracle."""
    B = bpm()
    # long marches in short rounds (about 50 rounds each), so all of them are
    # active together once admitted
    target_p, target_psi = synth.flat_bragg_scan(n_angles=1, nx=2048, nz=3000, precision="f32")[0]
    others = synth.flat_bragg_scan(n_angles=390, nx=1024, nz=3000, precision="f32")
    srv = B.Server(hbm_budget_bytes=4 << 30, max_slots=1024, chunk_steps=8)
    tick, copies = [], []
    for k, (p, psi) in enumerate(others):
        tick.append(srv.submit(p, psi))
        if k % 39 == 0:
            copies.append(srv.submit(target_p, target_psi))
    assert srv.drain(120.0)
    st = srv.stats()
    say("400 requests: completed", st["completed"], "launches", st["launches"])
    assert st["completed"] == len(tick) + len(copies) and st["failed"] == 0
    res = [srv.poll(t) for t in copies]
    for r in res:
        assert r["status"] == 0
        assert np.array_equal(r["psi_p"], res[0]["psi_p"]) and np.array_equal(r["psi_m"], res[0]["psi_m"])
        assert r["R"] == res[0]["R"] and r["T"] == res[0]["T"]
    op, om, oR, oT = oracle.propagate(target_p, target_psi)
    assert rel_pair(res[0]["psi_p"], res[0]["psi_m"], op, om) <= TOL["f32"][0]
    assert abs(res[0]["R"] - oR) <= r_bar("f32", oR) and abs(res[0]["T"] - oT) <= t_bar("f32", oT)
    for k in (0, 199, 389):
        p, psi = others[k]
        r = srv.poll(tick[k])
        op, om, oR, _ = oracle.propagate(p, psi)
        assert r["status"] == 0 and rel_pair(r["psi_p"], r["psi_m"], op, om) <= TOL["f32"][0]
    srv.close()


@pytest.mark.parametrize("order", [1, 2])
def test_server_zero_step_request_returns_entrance_state(order):
    """A request with nz = 0 through the server: the exit state is the entrance
    state and R, T are its detector powers (the server once ran one step)."""
    B = bpm()
    p = synth.base_problem(256, 0, 0.1, 0.05, synth.mask_empty(0), det=(40, 200), precision="f32")
    p["split_order"] = order
    a, b = synth.random_envelopes(256, 21)
    op, om, oR, oT = oracle.propagate(p, a, b)
    srv = B.Server(hbm_budget_bytes=1 << 30, max_slots=8, chunk_steps=16)
    t = srv.submit(p, a, b)
    assert srv.drain(60.0)
    r = srv.poll(t)
    srv.close()
    assert r is not None and r["status"] == 0
    assert rel_pair(r["psi_p"], r["psi_m"], op, om) <= TOL["f32"][0]
    assert abs(r["R"] - oR) <= r_bar("f32", oR) and abs(r["T"] - oT) <= t_bar("f32", oT)


def test_server_budget_and_cancel():
    B = bpm()
    p, psi = synth.flat_bragg_scan(n_angles=1, nx=1024, nz=200, precision="f32")[0]
    srv = B.Server(hbm_budget_bytes=64 * 1024, max_slots=4, chunk_steps=50)
    big = synth.flat_bragg_scan(n_angles=1, nx=8192, nz=10, precision="f64")[0]
    t_big = srv.submit(*big)
    r = srv.poll(t_big)
    assert r is not None and r["status"] == B.E_BUDGET
    ts = [srv.submit(p, psi) for _ in range(3)]
    assert srv.drain(60.0)
    res = [srv.poll(t) for t in ts]
    assert all(r["status"] == 0 for r in res)
    assert srv.stats()["peak_bytes"] <= 64 * 1024
    op, om, _, _ = oracle.propagate(p, psi)
    assert rel_pair(res[1]["psi_p"], res[1]["psi_m"], op, om) <= TOL["f32"][0]
    srv.close()


def test_server_cancel_stops_a_regular_lane_solve_early():
    """A request whose march takes seconds on one workgroup (resident size, no
    wide lane), cancelled 0.3 s after submission, completes with BPM_E_CANCELLED
    at the next round boundary, after a small part of its cell-steps; the
    requests beside it complete and match the oracle."""
    B = bpm()
    import time
    nz = 400000
    long_p = synth.base_problem(4096, nz, 0.1, 0.05, synth.mask_full(nz, 4096), precision="f32")
    long_psi = synth.gaussian_beam(4096, 0.1, 200.0, 20.0, 0.0)
    total = 2.0 * 4096 * nz
    p, psi = synth.flat_bragg_scan(n_angles=1, nx=1024, nz=200, precision="f32")[0]
    srv = B.Server(hbm_budget_bytes=1 << 30, max_slots=8, chunk_steps=64)
    t_long = srv.submit(long_p, long_psi, want_fields=False)
    ts = [srv.submit(p, psi) for _ in range(2)]
    time.sleep(0.3)
    t_cancel = time.perf_counter()
    srv.cancel(t_long)
    assert srv.drain(60.0)
    waited = time.perf_counter() - t_cancel
    r = srv.poll(t_long)
    st = srv.stats()
    done = st["cell_steps_done"] - 2 * 2.0 * 1024 * 200
    say("cancelled regular solve: status", r["status"], "its cell-steps %.3g of %.3g, drained %.2f s after cancel"
        % (done, total, waited))
    assert r["status"] == B.E_CANCELLED
    assert st["cancelled"] == 1 and st["completed"] == 2
    assert done < 0.5 * total and waited < 5.0
    op, om, _, _ = oracle.propagate(p, psi)
    for t in ts:
        x = srv.poll(t)
        assert x["status"] == 0 and rel_pair(x["psi_p"], x["psi_m"], op, om) <= TOL["f32"][0]
    srv.close()


def test_server_cancels_a_wide_lane_solve_between_rounds():
    """A long request marching in the wide lane stops at the next round
    boundary when cancelled; the server keeps serving the others."""
    B = bpm()
    import time
    long_p, long_psi = synth.flat_bragg_scan(n_angles=1, nx=65536, nz=200000, precision="f32")[0]
    short_p, short_psi = synth.flat_bragg_scan(n_angles=1, nx=2048, nz=300, precision="f32")[0]
    srv = B.Server(hbm_budget_bytes=4 << 30, max_slots=8, chunk_steps=256)
    t_long = srv.submit(long_p, long_psi, want_fields=False)
    time.sleep(0.3)   # a few rounds in (the whole march takes about 3 s wide, 70 s on one workgroup)
    srv.cancel(t_long)
    t_short = srv.submit(short_p, short_psi)
    assert srv.drain(60.0)
    r = srv.poll(t_long)
    st = srv.stats()
    say("cancelled wide solve: status", r["status"], "wide", st["wide"], "cell-steps done %.3g" % st["cell_steps_done"])
    assert r["status"] == B.E_CANCELLED and st["wide"] == 1
    assert st["cell_steps_done"] < 0.5 * 2.0 * 65536 * 200000
    x = srv.poll(t_short)
    assert x["status"] == 0
    op, om, _, _ = oracle.propagate(short_p, short_psi)
    assert rel_pair(x["psi_p"], x["psi_m"], op, om) <= TOL["f32"][0]
    srv.close()


def test_invalid_descriptors_rejected_before_any_launch():
    B = bpm()
    p, psi = synth.flat_bragg_scan(n_angles=1, nx=1024, nz=10)[0]
    for bad in ({"nx": 1000}, {"dz_um": -1.0}, {"lambda_um": 1.0}, {"det_hi": 5000}):
        with pytest.raises(B.BpmError) as e:
            B.Plan(dict(p, **bad))
        assert e.value.status == B.E_INVALID
    plan = B.Plan(p)
    bad = psi.copy()
    bad[7] = np.nan
    with pytest.raises(B.BpmError) as e:
        plan.propagate(bad)
    assert e.value.status == B.E_NUMERIC


# ------------------------------------------------------------------ staged FP32 lifting-form table, long march
def test_staged_fp32_lifting_table_long_march_random_fields():
    """The FP32 staged sizes hold P/N as an exact-angle lifting rotation; a
    fixed rounding in a table entry would add up linearly in Nz wherever the
    field has energy at large |P - 1|.  Random envelopes (energy in every bin)
    over 2000 steps at Nx 32768, through the staged batch kernel and the wide
    lane, against the oracle at the FP32 bars."""
    import torch
    B = bpm()
    nx, nz, dx, dz = 32768, 2000, 0.05, 0.025
    seg = np.zeros((nz, 1, 2), np.int32)
    for n in range(nz):
        seg[n, 0] = (nx // 16 + (n % 97), nx - nx // 9)
    p = synth.base_problem(nx, nz, dx, dz, seg, precision="f32", chih=CHIH_U, chihb=CHIHB_U)
    a, b = synth.random_envelopes(nx, 47)
    b = 0.5 * b
    op, om, oR, oT = oracle.propagate(p, a, b)
    tol = TOL["f32"][0]
    # wide lane (one solve alone)
    plan = B.Plan(p)
    gp, gm, gR, gT = plan.propagate(a, b)
    err = rel_pair(gp, gm, op, om)
    say("lifting long march, wide lane: rel L2 %.3e dR %.2e dT %.2e" % (err, abs(gR - oR), abs(gT - oT)))
    assert err <= tol and abs(gR - oR) <= r_bar("f32", oR) and abs(gT - oT) <= t_bar("f32", oT)
    # staged batch kernel (two copies of the solve in one launch)
    plans = [plan, B.Plan(p)]
    batch = B.Batch(plans)
    buf = batch.pack([(a, b), (a, b)])
    rt = torch.zeros(4, dtype=torch.float64, device="cuda")
    batch.run(buf.data_ptr(), buf.data_ptr(), rt.data_ptr())
    torch.cuda.synchronize()
    outs = batch.unpack(buf)
    rt = rt.cpu().numpy()
    batch.close()
    for q in plans:
        q.close()
    for i in range(2):
        err = rel_pair(outs[i][0], outs[i][1], op, om)
        say("lifting long march, batch %d: rel L2 %.3e dR %.2e dT %.2e" % (i, err, abs(rt[2 * i] - oR),
                                                                         abs(rt[2 * i + 1] - oT)))
        assert err <= tol and abs(rt[2 * i] - oR) <= r_bar("f32", oR) and abs(rt[2 * i + 1] - oT) <= t_bar("f32", oT)


# ------------------------------------------------------------------ POLY1: a polynomial phase without its X^2 term
def test_linear_phase_class_equals_the_polynomial_kernels_bitwise():
    """A bend (u = X Z / R, c3 = 0) runs the per-size FP32 kernels' POLY1 copy,
    whose phasor steps leave out the second-difference factor (exactly one for
    c3 = 0); the mixed-size and any-size kernels run the same solve as POLY2.
    The results must agree bitwise and match the oracle; a phase with an X^2
    term (c3 != 0) runs POLY2 everywhere."""
    import torch
    B = bpm()
    cases = []
    p, psi = synth.bent_laue(radii_m=(0.3,), nx=8192, nz=120, thickness=3.0, precision="f32")[0]
    cases.append((p, psi))
    q = dict(p, strain=dict(p["strain"], c=[0.0, 1e-5, 2e-7, -3e-9, p["strain"]["c"][4], 1e-9]))
    cases.append((q, psi))
    try:
        for k, (pp, ps) in enumerate(cases):
            op, om, oR, oT = oracle.propagate(pp, ps)
            outs = {}
            for sched in ("uniform", "mixed", "any"):
                B.schedule_set("f32", 8192, 1, sched)
                plan = B.Plan(pp)
                batch = B.Batch([plan])
                buf = batch.pack([(ps, None)])
                rt = torch.zeros(2, dtype=torch.float64, device="cuda")
                batch.run(buf.data_ptr(), buf.data_ptr(), rt.data_ptr())
                torch.cuda.synchronize()
                outs[sched] = batch.unpack(buf)[0]
                err = rel_pair(outs[sched][0], outs[sched][1], op, om)
                say("poly case %d schedule %s rel L2 %.3e" % (k, sched, err))
                assert err <= TOL["f32"][0] and abs(rt.cpu().numpy()[0] - oR) <= r_bar("f32", oR)
                batch.close()
                plan.close()
            for sched in ("mixed", "any"):
                assert np.array_equal(outs["uniform"][0], outs[sched][0]), (k, sched)
                assert np.array_equal(outs["uniform"][1], outs[sched][1]), (k, sched)
    finally:
        B.schedule_set("f32", 8192, 1, "default")
