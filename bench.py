#!/usr/bin/env python
"""Throughput of one fourth-order ADER-WENO-AO divergence-free MHD step on one
MI355X: zone-updates per second on a 6 x 128 x 128 angular x 128 radial
cube-based geodesic shell (12,582,912 zones, cubic isoparametric zones) with
a circularly polarised Alfven wave plus 1% seeded noise in density and
pressure (synthetic, seeded).  Prints one JSON line.

Timed region: K steps of the HIP library on device-resident state, bracketed
by torch.cuda.synchronize() and HIP events on the library's stream.  Mesh and
geometry construction and initial data are excluded (reported separately).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X vector FP64 (256 CU x 2.4 GHz x 128 flop/clk)
PEAK_HBM_GBS = 8000.0       # MI355X HBM3E
MACHINE_BALANCE = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


STAGE_KERNEL = {"bc_fill": "bc_zones", "weno": "weno_mfma<{p}>",
                "face_bnodal": "zone_face_bn<{p}, double>", "bmap": "bmap<{p}, double>",
                "predictor": "predictor<{p}, double, false>", "face_flux": "face_flux<{p}, double, false>",
                "edge_emf": "edge_emf<double, false>", "update_ct": "zone_update"}


KERNEL_SOURCES = ("step.hip", "mhd_device.hpp", "dtab.hpp")


def kernel_sources_sha256():
    """hash of the sources the step's kernels are compiled from"""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1905_02504_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, calibrated
    against a copy of known size) from the committed rocprofv3 summary, or None
    when the kernel sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_step_order4_6x128cubed.md")
    if not os.path.exists(path):
        return None
    sha = kernel_sources_sha256()
    head = f"traffic {kernel} "
    for line in open(path):
        if line.startswith(head):
            kv = dict(t.split("=", 1) for t in line[len(head):].split())
            if kv.get("kernel_sources_sha256") != sha:
                return None
            return float(kv["read_bytes"]) + float(kv["write_bytes"])
    return None


def host_cpu_model():
    """The host CPU's model name and logical CPU count (lscpu, else /proc/cpuinfo)."""
    import subprocess
    model, cpus = None, os.cpu_count()
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() == "Model name":
                model = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return {"model": model, "logical_cpus": cpus}


def cpu_baseline(order, sample_n=16, sample_nr=16):
    """The oracle, as it stands, on a bounded sample of the same workload, on
    all the OpenMP threads it gets, and on one thread for a smaller sample."""
    import ctypes
    import numpy as np
    import rg_inputs as RI
    from oracle import oracle as O
    prob = RI.alfven_problem()

    def one_step(n, nr):
        m = O.OracleMesh(n, nr, order=order, n_ghost=order - 1)
        U, Bf = m.init_alfven(prob)
        noise = RI.white_noise(m.nz)
        U[0] *= 1 + 0.01 * noise[0]
        dt = m.cfl_dt(U, 0.3, prob["gamma"])
        t0 = time.perf_counter()
        m.step(U, Bf, dt, gamma=prob["gamma"])
        return time.perf_counter() - t0, 6 * n * n * nr

    def c1_step(n):
        """one third-order step of the multi-harmonic state on 6 x n^3 zones"""
        m = O.OracleMesh(n, n, order=3, n_ghost=2)
        hp = RI.harmonic_problem()
        U, Bf = m.init_harmonic(hp)
        dt = m.cfl_dt(U, 0.4, hp["gamma"])
        t0 = time.perf_counter()
        m.step(U, Bf, dt, gamma=hp["gamma"])
        return time.perf_counter() - t0, 6 * n ** 3

    def c4_gradient():
        """one directional derivative of a third-order step on 6 x 8^3 zones by
        the oracle's complex step (the oracle gradient of the adjoint checks)"""
        m = O.OracleMesh(8, 8, order=3, n_ghost=2)
        U, Bf = m.init_alfven(prob)
        dt = m.cfl_dt(U, 0.3, prob["gamma"])
        d = np.random.default_rng(5).uniform(-1, 1, U.shape)
        t0 = time.perf_counter()
        m.step_complex(U + 1e-30j * d, Bf.astype(np.complex128), dt, gamma=prob["gamma"])
        return time.perf_counter() - t0, 6 * 8 ** 3

    O.lib()   # the oracle's OpenMP runtime is the process's libgomp
    gomp = ctypes.CDLL("libgomp.so.1")
    threads = gomp.omp_get_max_threads()
    el, zones = one_step(sample_n, sample_nr)
    elc1, zc1 = c1_step(16)
    elg, zg = c4_gradient()
    gomp.omp_set_num_threads(1)
    try:
        el1, zones1 = one_step(4, 8)
        elc1_1, zc1_1 = c1_step(8)
        elg1, _ = c4_gradient()
    finally:
        gomp.omp_set_num_threads(threads)
    return {"value": zones / el, "unit": "zone-updates/s", "cores": threads, "kind": "oracle",
            "host_cpu": host_cpu_model(),
            "sample": f"one order-{order} step on 6x{sample_n}x{sample_n}x{sample_nr} zones "
                      f"(Alfven wave + noise), {el:.2f} s, geometry excluded",
            "single_thread": {"value": zones1 / el1, "sample": f"one order-{order} step on 6x4x4x8 zones, "
                                                                f"{el1:.2f} s"},
            "order3": {"all_threads": zc1 / elc1, "single_thread": zc1_1 / elc1_1, "unit": "zone-updates/s",
                       "sample": "one third-order step of the multi-harmonic state, 6x16^3 zones on all threads, "
                                 "6x8^3 on one"},
            "gradient_6x8cubed": {"all_threads": zg / elg, "single_thread": zg / elg1, "unit": "zone-updates/s",
                                  "sample": "one directional derivative of a third-order step by complex step"}}


def time_adjoint(reps=5):
    """Forward step and its adjoint (rg_step_adjoint, forward recomputation
    included) on the differentiation workload: third order, 6 x 32 x 32 x 32
    zones, Alfven wave + 1% noise, fixed dt; the FP64 step and the FP32 form.
    HIP events on the stream the library runs on."""
    import torch
    import paper_1905_02504_amd as R
    from paper_1905_02504_amd import _native as NV
    import rg_inputs as RI
    prob = RI.alfven_problem()
    gam = prob["gamma"]
    stream = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out, dt = [], None
    for mode in (NV.RG_MODE_FP64, NV.RG_MODE_FP32):
        sh = R.ShellMHD(32, 32, 3, n_ghost=2, mode=mode)
        U_h, Bf_h = sh.init_alfven(prob, noise=RI.white_noise(sh.nz), noise_amp=0.01)
        U, Bf = torch.from_numpy(U_h).cuda(), torch.from_numpy(Bf_h).cuda()
        if dt is None:
            dt = sh.cfl_dt(U, 0.4, gam)
        gen = torch.Generator(device="cuda").manual_seed(7)
        gU1 = torch.rand(U.shape, dtype=torch.float64, device="cuda", generator=gen)
        gB1 = torch.rand(Bf.shape, dtype=torch.float64, device="cuda", generator=gen)
        U1, B1 = torch.empty_like(U), torch.empty_like(Bf)
        gU, gB = torch.empty_like(U), torch.empty_like(Bf)
        t_fwd = timed(lambda: sh.step(U, Bf, dt, gamma=gam, U_out=U1, Bf_out=B1))
        t_adj = timed(lambda: sh.step_adjoint(U, Bf, gU1, gB1, dt, gamma=gam, gU=gU, gBf=gB))
        if not (torch.isfinite(gU).all() and torch.isfinite(gB).all()):
            raise RuntimeError("non-finite adjoint")
        out.append((t_fwd, t_adj, gU, gB))
        sh.close()
    (t_fwd, t_adj, gU, gB), (t_fwd32, t_adj32, gU32, gB32) = out
    interior = 6 * 32 * 32 * 32
    return {"workload": "third order, 6x32x32 angular x 32 radial = 196608 zones, Alfven wave + 1% noise, "
                        "fixed dt; adjoint includes its recomputation of the step up to the predictor",
            "ms_per_step": t_fwd, "ms_per_adjoint": t_adj, "adjoint_over_step": t_adj / t_fwd,
            "adjoint_zone_updates_per_s": interior / (t_adj * 1e-3),
            "fp32": {"ms_per_step": t_fwd32, "ms_per_adjoint": t_adj32, "adjoint_speedup_vs_fp64": t_adj / t_adj32,
                     "rel_l2_vs_fp64_adjoint": {"zone_state": float((gU32 - gU).norm() / gU.norm()),
                                                "face_B": float((gB32 - gB).norm() / gB.norm())}}}


def time_prism(level=6, n_rad=128, order=4, reps=5):
    """The prism element's ADER-CG predictor (rg_prism_predict) on the
    icosahedral geodesic mesh: fourth order, level 6 (81,920 spherical
    triangles, mean edge 1.08 degrees: a quarter of the sphere of the paper's
    finest 0.54-degree, 128-shell mesh, one GPU's share) x 128 logarithmic
    shells, 10.5 M zones; uniform state with 5 % seeded noise, dt 2e-3.  HIP
    events on the stream the library runs on."""
    import torch
    import paper_1905_02504_amd as R
    lib = R.PrismMesh(level, n_rad, order, r_in=1.0, r_out=2.0)
    gen = torch.Generator(device="cuda").manual_seed(7)
    base = torch.tensor([1.0, 0.3, -0.2, 0.1, 2.0, 0.4, 0.2, -0.3], dtype=torch.float64, device="cuda")
    Ua = base[:, None, None] * (1 + 0.05 * (2 * torch.rand((8, lib.nz, lib.N), generator=gen, device="cuda",
                                                             dtype=torch.float64) - 1))
    aU = torch.empty_like(Ua)
    aF = torch.empty((3, 8, lib.nz, lib.N), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(2):
        lib.predict(Ua, 2e-3, aU=aU, aF=aF)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        lib.predict(Ua, 2e-3, aU=aU, aF=aF)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    if not (torch.isfinite(aU).all() and torch.isfinite(aF).all()):
        raise RuntimeError("non-finite prism predictor output")
    # face traces at the rules of Appendix A (HBM-bound: 32 N values read and
    # 32 Q written per zone)
    del Ua
    tr = torch.empty((32, lib.Q, lib.nz), dtype=torch.float64, device="cuda")
    lib.traces(aU, aF, tr)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        lib.traces(aU, aF, tr)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_tr = e0.elapsed_time(e1) / reps
    tr_bytes = 8.0 * 32 * (lib.N + lib.Q)
    # HLL face fluxes of every radial and side face from the traces
    Phi = torch.empty((lib.n_faces, 8), dtype=torch.float64, device="cuda")
    lib.face_fluxes(tr, Phi=Phi)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        lib.face_fluxes(tr, Phi=Phi)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_ff = e0.elapsed_time(e1) / reps
    if not torch.isfinite(Phi).all():
        raise RuntimeError("non-finite prism face fluxes")
    n_faces = lib.n_faces
    ff_bytes = 8.0 * (32 * lib.Q * lib.nz + 8 * n_faces)
    # finite-volume update of the zone averages from the face fluxes
    U = base[:, None] * (1 + 0.05 * (2 * torch.rand((8, lib.nz), generator=gen, device="cuda",
                                                     dtype=torch.float64) - 1))
    U1 = torch.empty_like(U)
    lib.update(U, Phi, 2e-3, U1)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        lib.update(U, Phi, 2e-3, U1)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_up = e0.elapsed_time(e1) / reps
    up_bytes = 8.0 * (16 * lib.nz + 5 * 8 * lib.nz)
    del U, U1
    # constrained transport: the predictor's averages at the edge points,
    # the edge integrals of E, then the face magnetic fluxes
    er = lib.edge_traces(aU, aF)
    Ga, Gr = lib.edge_emfs(er)
    PhiB = torch.zeros(lib.n_faces, dtype=torch.float64, device="cuda")
    PhiB1 = lib.ct(PhiB, Ga, Gr, 2e-3)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        lib.edge_traces(aU, aF, er)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_etr = e0.elapsed_time(e1) / reps
    e0.record(stream)
    for _ in range(reps):
        lib.edge_emfs(er, Gang=Ga, Grad=Gr)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_emf = e0.elapsed_time(e1) / reps
    e0.record(stream)
    for _ in range(reps):
        lib.ct(PhiB, Ga, Gr, 2e-3, out=PhiB1)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_ct = e0.elapsed_time(e1) / reps
    if not (torch.isfinite(Ga).all() and torch.isfinite(Gr).all() and torch.isfinite(PhiB1).all()):
        raise RuntimeError("non-finite prism edge fields")
    n_aedges, n_redges = Ga.numel(), Gr.numel()
    del er, Ga, Gr, PhiB, PhiB1
    # divergence-free reconstruction of B: one column map per column applied
    # to every shell (the first call builds and uploads the maps, untimed)
    nin, nout = lib.n_divfree_in, lib.n_divfree_out
    Bin = torch.randn((nin, lib.nz), generator=gen, device="cuda", dtype=torch.float64)
    Bout = torch.empty((nout, lib.nz), dtype=torch.float64, device="cuda")
    t_maps = time.perf_counter()
    lib.divfree(Bin, Bout)
    torch.cuda.synchronize()
    t_maps = time.perf_counter() - t_maps
    e0.record(stream)
    for _ in range(reps):
        lib.divfree(Bin, Bout)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_df = e0.elapsed_time(e1) / reps
    if not torch.isfinite(Bout).all():
        raise RuntimeError("non-finite divergence-free reconstruction")
    df_bytes = 8.0 * (nin + nout) + 8.0 * nin * nout / n_rad     # per zone: in, out, the column's map shared by its shells
    df_flops = 2.0 * nin * nout
    del Bin, Bout
    flops, nbytes = lib.work()
    nz, lib_q, lib_n = lib.nz, lib.Q, lib.N
    del aU, aF, tr, Phi
    lib.close()
    torch.cuda.empty_cache()
    tf = flops * nz / (ms * 1e-3) / 1e12
    chain_ms = ms + ms_tr + ms_ff + ms_up + ms_etr + ms_emf + ms_ct + ms_df
    return {"workload": f"prism ADER-CG predictor, order {order}, icosahedral level {level} "
                        f"({20 * 4 ** level} triangles) x {n_rad} shells = {nz} zones, uniform state + 5% noise",
            "zones": nz, "ms_per_predictor": ms, "zone_updates_per_s": nz / (ms * 1e-3),
            "flops_per_zone": flops, "bytes_per_zone": nbytes,
            "traces": {"ms": ms_tr, "face_points_per_zone": lib_q, "bytes_per_zone": tr_bytes,
                       "hbm_gbs": tr_bytes * nz / (ms_tr * 1e-3) / 1e9},
            "face_fluxes": {"ms": ms_ff, "faces": n_faces, "face_updates_per_s": n_faces / (ms_ff * 1e-3),
                            "hbm_gbs": ff_bytes / (ms_ff * 1e-3) / 1e9},
            "update": {"ms": ms_up, "hbm_gbs": up_bytes / (ms_up * 1e-3) / 1e9},
            "edge_traces": {"ms": ms_etr, "hbm_gbs": 8.0 * 17 * (lib_n + 27) * nz / (ms_etr * 1e-3) / 1e9},
            "edge_emfs": {"ms": ms_emf, "angular_edges": n_aedges, "radial_edges": n_redges},
            "ct": {"ms": ms_ct},
            "divfree": {"ms": ms_df, "inputs": nin, "outputs": nout, "bytes_per_zone": df_bytes,
                        "flops_per_zone": df_flops, "hbm_gbs": df_bytes * nz / (ms_df * 1e-3) / 1e9,
                        "tflops": df_flops * nz / (ms_df * 1e-3) / 1e12, "map_build_s": t_maps},
            "roofline": {"bound": "alu", "achieved": tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                         "frac": tf / PEAK_FP64_TFLOPS, "hbm_gbs": nbytes * nz / (ms * 1e-3) / 1e9},
            # the built stages of one prism step in sequence (the WENO-AO
            # reconstruction on triangle stencils, which would feed the
            # predictor and the divergence-free map, is not built)
            "chain_without_reconstruction": {
                "ms": chain_ms, "zone_updates_per_s": nz / (chain_ms * 1e-3),
                "stages": "predictor, face traces, face fluxes, update, edge traces, edge fields, CT, divergence-free B"}}


def measured_peaks(reps=5):
    """Attainable rates on this GPU, beside the datasheet peaks: the FP64
    vector FMA rate of rg_fma_probe (16 independent chains per lane), the FP64
    and BF16 matrix-core rates of rg_mfma_probe (8 independent products per
    wavefront) and the bandwidth of a 2 GiB device-to-device copy (bytes read +
    written)."""
    import torch
    from paper_1905_02504_amd import _native as NV
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    n, iters = 256 * 8192, 2048
    sink = torch.empty(n, dtype=torch.float64, device="cuda")
    t = timed(lambda: NV.rg_fma_probe(sink.data_ptr(), n, iters, stream.cuda_stream))
    fp64 = 2.0 * 16 * iters * n / t / 1e12
    # matrix cores: eight independent products per wavefront and iteration
    nm, im = 256 * 4096, 256
    t = timed(lambda: NV.rg_mfma_probe(sink.data_ptr(), nm, im, 0, stream.cuda_stream))
    mfma64 = 2048.0 * 8 * im * (nm // 64) / t / 1e12
    t = timed(lambda: NV.rg_mfma_probe(sink.data_ptr(), nm, 4 * im, 1, stream.cuda_stream))
    mfma_bf16 = 16384.0 * 8 * 4 * im * (nm // 64) / t / 1e12
    del sink
    a = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    t = timed(lambda: b.copy_(a))
    gbs = 2.0 * a.numel() * 8 / t / 1e9
    del a, b
    return {"fp64_valu_tflops": fp64, "fp64_mfma_tflops": mfma64, "bf16_mfma_tflops": mfma_bf16, "hbm_copy_gbs": gbs}


def weno_order_stats(sh):
    """Summary of the last step's WENO-AO order indicator over the interior
    zones (the large stencil's weight over its linear weight, smallest over
    the variables)."""
    import torch
    w = sh.weno_order()[torch.from_numpy(sh.interior()).cuda()].double()
    return {"min": float(w.min()), "median": float(w.median()), "frac_below_0.5": float((w < 0.5).double().mean()),
            "frac_below_0.01": float((w < 0.01).double().mean())}


def time_blast(n_steps=50, mode=0):
    """The magnetised blast (p = 1000 in a ball of radius 0.1 at 1.5 a, beta
    0.025 outside) on 6 x 96^2 x 96 = 5,308,416 zones, fourth order, with the
    first-order fallback, dt from CFL 0.15 every step (its reduction and host
    read are in the timed loop, as is a device-side count of the flagged
    zones); zone averages by cubature of the pressure step (rg_init_blast).
    mode 0: the FP64 scheme, 1: the FP32 form."""
    import torch
    import paper_1905_02504_amd as R
    import rg_inputs as RI
    sh = R.ShellMHD(96, 96, 4, n_ghost=3, mode=mode)
    prob = RI.blast_problem(p_in=1000.0, radius=0.1)
    gam = prob["gamma"]
    U_h, Bf_h = sh.init_blast(prob)
    U, Bf = torch.from_numpy(U_h).cuda(), torch.from_numpy(Bf_h).cuda()
    del U_h, Bf_h
    U2, Bf2 = torch.empty_like(U), torch.empty_like(Bf)
    flagged = torch.zeros((), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_sim = 0.0
    for _ in range(n_steps):
        _, _, dt = sh.step(U, Bf, 0.0, gamma=gam, cfl=0.15, U_out=U2, Bf_out=Bf2, fallback=True)
        flagged += sh.fallback_zones().sum()
        t_sim += dt
        U, U2, Bf, Bf2 = U2, U, Bf2, Bf
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / n_steps * 1e3
    d = sh.diag(U, Bf, gam)
    wo = weno_order_stats(sh)
    interior = 6 * 96 * 96 * 96
    sh.close()
    return {"workload": "magnetised blast, order 4, 6x96x96 angular x 96 radial = 5308416 zones, "
                        f"{n_steps} steps at CFL 0.15 with the first-order fallback, "
                        + ("FP64 scheme" if mode == 0 else "FP32 form"),
            "ms_per_step": ms, "zone_updates_per_s": interior / (ms * 1e-3), "t_final": t_sim,
            "fallback_zone_steps": int(flagged.item()), "rho_min": d["rho_min"], "p_min": d["p_min"],
            "div_b_rel_max": d["div_rel_max"], "weno_order_last_step": wo}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-ang", type=int, default=128)
    ap.add_argument("--n-rad", type=int, default=128)
    ap.add_argument("--order", type=int, default=4)
    ap.add_argument("--cfl", type=float, default=0.3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32-form run")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timing")
    ap.add_argument("--no-blast", action="store_true", help="skip the magnetised-blast run")
    ap.add_argument("--no-fallback", action="store_true", help="skip the timing with the fallback on")
    ap.add_argument("--no-prism", action="store_true", help="skip the prism-element predictor timing")
    ap.add_argument("--calib", action="store_true",
                    help="run a 1 GiB device-to-device copy first (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the step is one GPU's share of the mesh); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1905_02504_amd as R
    import rg_inputs as RI

    t0 = time.perf_counter()
    shell = R.ShellMHD(args.n_ang, args.n_rad, args.order, n_ghost=max(3, args.order - 1))
    t_geom = time.perf_counter() - t0
    log(f"[bench] geometry {t_geom:.1f}s, zones {shell.nz}")
    prob = RI.alfven_problem()
    t0 = time.perf_counter()
    noise = RI.white_noise(shell.nz)
    U_h, Bf_h = shell.init_alfven(prob, noise=noise, noise_amp=0.01)
    t_init = time.perf_counter() - t0
    log(f"[bench] initial data {t_init:.1f}s")
    U0 = torch.from_numpy(U_h).cuda()
    Bf0 = torch.from_numpy(Bf_h).cuda()
    del U_h, Bf_h, noise
    gam = prob["gamma"]
    if args.calib:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("[bench] calibration copy: 1 GiB read + 1 GiB written")
    dt = shell.cfl_dt(U0, args.cfl, gam)

    def run(sh, fallback=False):
        """warmup + timed steps from the initial state; returns the final state"""
        U, Bf = U0.clone(), Bf0.clone()
        U2, Bf2 = torch.empty_like(U), torch.empty_like(Bf)
        for _ in range(args.warmup):
            sh.step(U, Bf, dt, gamma=gam, U_out=U2, Bf_out=Bf2, fallback=fallback)
            U, U2, Bf, Bf2 = U2, U, Bf2, Bf
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        sh.profile_begin()
        ev0.record(stream)
        for _ in range(args.steps):
            sh.step(U, Bf, dt, gamma=gam, U_out=U2, Bf_out=Bf2, fallback=fallback)
            U, U2, Bf, Bf2 = U2, U, Bf2, Bf
        ev1.record(stream)
        torch.cuda.synchronize()
        stage_ms, nrec = sh.profile_end()
        del U2, Bf2
        return U, Bf, ev0.elapsed_time(ev1), stage_ms, nrec

    U, Bf, total_ms, stage_ms, nrec = run(shell)
    ms_step = total_ms / args.steps
    interior = 6 * args.n_ang * args.n_ang * args.n_rad
    value = interior * args.steps / (total_ms * 1e-3)
    log(f"[bench] {ms_step:.2f} ms/step, stages (ms/step): " +
        ", ".join(f"{k} {v / nrec:.2f}" for k, v in stage_ms.items()))
    if not torch.isfinite(U).all():
        log("[bench] non-finite state after the timed steps")
        sys.exit(1)
    diag64 = shell.diag(U, Bf, gam)
    weno_order = weno_order_stats(shell)
    log(f"[bench] FP64: max relative div B {diag64['div_rel_max']:.2e}, "
        f"min rho {diag64['rho_min']:.4f}, min p {diag64['p_min']:.4f}")

    # the same steps with the first-order fallback on (smooth data: the checks
    # run, nothing is flagged): the cost of its passes
    fallback = None
    if not args.no_fallback:
        Ufb, _, total_fb, stage_fb, nrec_fb = run(shell, fallback=True)
        nflag = int(shell.fallback_zones().sum().item())
        fallback = {"ms_per_step": total_fb / args.steps, "overhead_vs_plain": total_fb / total_ms - 1.0,
                    "update_ct_stage_ms": stage_fb["update_ct"] / nrec_fb, "zones_flagged_last_step": nflag,
                    "state_equals_plain": bool(torch.equal(Ufb, U))}
        del Ufb
        log(f"[bench] with the fallback on: {fallback['ms_per_step']:.2f} ms/step "
            f"({100 * fallback['overhead_vs_plain']:.1f} % more), {nflag} zones flagged")

    flops, bytes_ = shell.work()
    dom = max(stage_ms, key=stage_ms.get)
    dom_s = stage_ms[dom] / nrec * 1e-3
    intensity = flops[dom] / max(bytes_[dom], 1.0)
    kname = STAGE_KERNEL[dom].format(p=args.order)
    traffic = measured_traffic(kname) if (args.n_ang, args.n_rad, args.order) == (128, 128, 4) else None
    if intensity >= MACHINE_BALANCE:
        achieved = flops[dom] / dom_s / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic, "kernel": kname,
                "algorithmic_flops": flops[dom], "algorithmic_bytes": bytes_[dom]}
    else:
        achieved = bytes_[dom] / dom_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "kernel": kname,
                "algorithmic_flops": flops[dom], "algorithmic_bytes": bytes_[dom]}
    peaks = measured_peaks()
    roof["measured_peak"] = peaks["fp64_valu_tflops"] if roof["unit"] == "TFLOP/s" else peaks["hbm_copy_gbs"]
    roof["frac_of_measured_peak"] = roof["achieved"] / roof["measured_peak"]
    if traffic is not None:
        roof["traffic_gbs"] = traffic / dom_s / 1e9   # measured HBM bytes over the kernel's time
    # the matrix-core stages: algorithmic flops over their time, against the
    # datasheet and the measured FP64 matrix-core rates
    mfma_stages = {}
    for st in ("weno", "bmap"):
        tf = flops[st] / (stage_ms[st] / nrec * 1e-3) / 1e12
        mfma_stages[st] = {"kernel": STAGE_KERNEL[st].format(p=args.order), "ms": stage_ms[st] / nrec,
                           "tflops": tf, "frac_of_peak": tf / PEAK_FP64_TFLOPS,
                           "frac_of_measured_mfma_peak": tf / peaks["fp64_mfma_tflops"]}
    log(f"[bench] measured peaks: FP64 FMA {peaks['fp64_valu_tflops']:.1f} TFLOP/s, FP64 MFMA "
        f"{peaks['fp64_mfma_tflops']:.1f} TFLOP/s, BF16 MFMA {peaks['bf16_mfma_tflops']:.0f} TFLOP/s, device copy "
        f"{peaks['hbm_copy_gbs']:.0f} GB/s; dominant kernel at {100 * roof['frac_of_measured_peak']:.1f} % of the "
        f"measured peak")
    mixed = None
    if not args.no_mixed:
        from paper_1905_02504_amd import _native as NV
        inter = torch.from_numpy(shell.interior()).cuda()
        shell.close()   # its work buffers and those of the FP32 geometry do not both fit in HBM
        names = ["rho", "mx", "my", "mz", "E", "Bx", "By", "Bz"]
        mixed = {}
        for tag, mode, what in (
                ("fp32", NV.RG_MODE_FP32, "fp32 (reconstruction, predictor and traces; geometry, div-free map, "
                                          "Riemann solvers, update and CT in fp64)"),
                ("bf16", NV.RG_MODE_BF16, "the fp32 form with the predictor's flux derivatives on the BF16 matrix "
                                          "cores (each fp32 value split exactly into three bf16 parts, fp32 "
                                          "accumulation)")):
            t0 = time.perf_counter()
            shell32 = R.ShellMHD(args.n_ang, args.n_rad, args.order, n_ghost=max(3, args.order - 1), mode=mode)
            log(f"[bench] {tag}-form geometry {time.perf_counter() - t0:.1f}s")
            U32, Bf32, total32, stage32, nrec32 = run(shell32)
            ms32 = total32 / args.steps
            log(f"[bench] {tag} form: {ms32:.2f} ms/step, stages (ms/step): " +
                ", ".join(f"{k} {v / nrec32:.2f}" for k, v in stage32.items()))
            a64, a32 = U[:, inter], U32[:, inter]
            l1 = ((a32 - a64).abs().sum(1) / a64.abs().sum(1)).cpu().numpy()
            l1b = float((Bf32 - Bf).abs().sum() / Bf.abs().sum())
            diag32 = shell32.diag(U32, Bf32, gam)
            mixed[tag] = {"mode": what,
                          "value": interior * args.steps / (total32 * 1e-3), "ms_per_step": ms32,
                          "speedup_vs_fp64": ms_step / ms32,
                          "rel_l1_vs_fp64_after_steps": args.warmup + args.steps,
                          "rel_l1_vs_fp64": {k: float(v) for k, v in zip(names, l1)}, "rel_l1_face_B": l1b,
                          "div_b_rel_max": diag32["div_rel_max"],
                          "stage_ms_per_step": {k: round(v / nrec32, 4) for k, v in stage32.items()}}
            del U32, Bf32
            shell32.close()
    adjoint = None
    if not args.no_adjoint:
        if args.no_mixed:
            shell.close()   # (the FP32 run closed it otherwise)
        adjoint = time_adjoint()
        log(f"[bench] adjoint (order 3, 6x32^3): step {adjoint['ms_per_step']:.2f} ms, "
            f"adjoint {adjoint['ms_per_adjoint']:.2f} ms ({adjoint['adjoint_over_step']:.1f}x); FP32 form: "
            f"step {adjoint['fp32']['ms_per_step']:.2f} ms, adjoint {adjoint['fp32']['ms_per_adjoint']:.2f} ms")
    blast = None
    if not args.no_blast:
        shell.close()
        blast = time_blast(mode=0)
        log(f"[bench] blast (order 4, 6x96^3, FP64): {blast['ms_per_step']:.2f} ms/step, "
            f"{blast['fallback_zone_steps']} fallback zone-steps, min rho {blast['rho_min']:.4f}, "
            f"min p {blast['p_min']:.3e}")
        blast["fp32"] = time_blast(mode=1)
        log(f"[bench] blast (order 4, 6x96^3, FP32 form): {blast['fp32']['ms_per_step']:.2f} ms/step, "
            f"{blast['fp32']['fallback_zone_steps']} fallback zone-steps, min rho {blast['fp32']['rho_min']:.4f}, "
            f"min p {blast['fp32']['p_min']:.3e}")
    prism = None
    if not args.no_prism:
        shell.close()   # the prism arrays (about 90 GB) need the HBM the step's buffers hold
        prism = time_prism()
        log(f"[bench] prism predictor (order 4, icosahedral level 6 x 128 = {prism['zones']} zones): "
            f"{prism['ms_per_predictor']:.2f} ms, {prism['zone_updates_per_s'] / 1e6:.1f} M zone-updates/s, "
            f"{prism['roofline']['achieved']:.1f} TFLOP/s ({100 * prism['roofline']['frac']:.1f} % of FP64 peak); "
            f"face traces {prism['traces']['ms']:.2f} ms ({prism['traces']['hbm_gbs']:.0f} GB/s), "
            f"face fluxes {prism['face_fluxes']['ms']:.2f} ms ({prism['face_fluxes']['hbm_gbs']:.0f} GB/s), "
            f"update {prism['update']['ms']:.2f} ms, edge traces {prism['edge_traces']['ms']:.2f} ms, "
            f"edge fields {prism['edge_emfs']['ms']:.2f} ms, "
            f"CT {prism['ct']['ms']:.2f} ms, divergence-free B {prism['divfree']['ms']:.2f} ms "
            f"({prism['divfree']['hbm_gbs']:.0f} GB/s, {prism['divfree']['tflops']:.1f} TFLOP/s; maps built in "
            f"{prism['divfree']['map_build_s']:.1f} s); these stages in sequence "
            f"{prism['chain_without_reconstruction']['ms']:.1f} ms = "
            f"{prism['chain_without_reconstruction']['zone_updates_per_s'] / 1e6:.1f} M zone-updates/s (no reconstruction)")
    out = {
        "metric": "zone-updates/s per ADER step (4th order), FP64",
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"ADER-WENO-AO MHD step, order {args.order}, 6x{args.n_ang}x{args.n_ang} angular x "
                               f"{args.n_rad} radial = {interior} zones, Alfven wave + 1% noise, CFL {args.cfl}",
                   "zones": interior, "order": args.order, "dt": dt,
                   "setup_s": {"geometry": round(t_geom, 2), "initial_data": round(t_init, 2)},
                   "stage_ms_per_step": {k: round(v / nrec, 4) for k, v in stage_ms.items()}},
        "roofline": roof,
        "mfma_stages": mfma_stages,
        "measured_peaks": peaks,
        "div_b_rel_max": diag64["div_rel_max"],
        "weno_order_last_step": weno_order,
        "mixed": mixed,
        "adjoint": adjoint,
        "fallback": fallback,
        "blast": blast,
        "prism": prism,
    }
    if not args.no_cpu_baseline:
        log("[bench] CPU baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline(args.order)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
