"""Benchmark: lattice H-matrix-vector products per second on one MI355X.

Workload: planar 30-degree dipping thrust fault of 480 x 256 squares of 50 m
(N = 122880), full-space coplanar kernel (mu = 32 GPa, nu = 0.25), ACA
eps = 1e-5, leaf 64, eta = 2, lattice 32 x 32; slip rates log-uniform in
[1e-12, 1e-9] m/s from seed 2.  One step is one H-matrix-vector product
y = H x (gather through the cluster permutation, dense near-field blocks,
both low-rank phases, row-owned accumulation, scatter back).

The headline value is the FP32-stored / FP64-accumulated batched product;
the plain FP64 product and the batched FP64 product are timed beside it.
Further sections of the same JSON line (each can be skipped by a flag):
construction (host and device), autotuner, size and lattice sweeps, a
1000-step RK45 run at N = 122880, the 64-member MFMA ensemble product
(curved thrust of 21000 triangles and the N = 122880 fault), the nonplanar
fault (A and B products, RK45 with sigma evolving), the 64-member ensemble
integration and the adjoint gradient on the curved thrust (A and B), and
the oracle's CPU rates on bounded samples (block loop, sparse form, exact
FFT product, Runge-Kutta steps).

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H-matvec/s and % of HBM peak at N≈1.2e5, FP32-batched vs FP64-plain, rel err ≤2e-5"
WORKLOAD = "dip30_480x256"
HBM_PEAK_GBS = 8000.0


# Dominant kernel of each schedule (launch index -> kernel symbol of the FP32 build).
DOMINANT_SYMBOL = {
    ("split", 1): "k_phase<float, 8, 2> (phase 2: y = D x + U t)",
    ("split", 0): "k_phase<float, 4, 1> (phase 1: t = V^T x)",
    ("persistent", 0): "k_persistent<float, 4>",
    ("plain", 1): "k_plain_p2<float>",
    ("plain", 0): "k_plain_p1<float>",
}
# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE counters, each scaled by what
# the counter reads for a 1 GiB device copy (profiles/k_phase_dip30_480x256_counters.md),
# keyed by the hash of the kernel and layout sources they were taken with: any change to
# those sources makes the entry inapplicable (traffic reported as null until re-measured).
TRAFFIC = {
    ("split", 1, "9a6f662e5ae6d66e"): 870710630,
    ("split", 0, "9a6f662e5ae6d66e"): 593387757,
}
TRAFFIC_SOURCES = ("paper_2110_12165_amd/csrc/kernels.hip", "paper_2110_12165_amd/csrc/layout.cpp",
                   "paper_2110_12165_amd/csrc/device_types.hpp")


def source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_products(torch, H, x, y, steps, warmup):
    """Returns (ms per product over the timed region, mean launch duration in ms
    from per-product HIP events on the launch stream)."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        H.matvec(x, y=y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        H.matvec(x, y=y)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    region = ev0.elapsed_time(ev1) / steps
    # per-launch durations: each product bracketed by its own events
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in evs:
        a.record(stream)
        H.matvec(x, y=y)
        b.record(stream)
    torch.cuda.synchronize()
    per = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    return max(region, 1e-9), per, wall


def _timed(fn, seconds):
    """Seconds per call of fn over about `seconds` (after one untimed call)."""
    fn()
    reps, t0 = 0, time.perf_counter()
    while True:
        out = fn()
        reps += 1
        el = time.perf_counter() - t0
        if el > seconds:
            return el / reps, reps, el, out


def cpu_baseline(f, w, x, y_gpu):
    """The oracle timed on the host cores, on bounded samples:

    * the H-matrix product on the complete lattice block-rows 0 and 15 (2 of
      32, 7680 of 122880 rows), built by the oracle's own ACA, scaled to
      full products by the row fraction: the block loop with all host
      threads for BLAS (the headline value) and with one thread, and the
      sparse form (SciPy CSR) with one thread and with row chunks on all
      host threads;
    * the exact product of the whole matrix by FFT (the dense definition,
      N = 122880; NumPy's FFT runs on one thread);
    * the oracle's Runge-Kutta integration on the 2048-element fault
      (steps per second, block-loop product)."""
    from threadpoolctl import threadpool_limits

    from oracle import friction as fr
    from oracle import rk45 as ork
    from oracle.dense import fft_grid_product
    from oracle.greens import CoplanarRectGeometry
    from oracle.hmatrix import HMatrix as OracleH
    from oracle.hmatrix import SparseHMatrix
    from synth import WORKLOADS, config_fault, friction_params
    from synth.faults import MU, NU

    threads = len(os.sched_getaffinity(0))
    g = CoplanarRectGeometry(f.verts, f.slip_dir, MU, NU)
    rows_sel = (0, 15)
    t0 = time.perf_counter()
    with threadpool_limits(limits=threads):
        H = OracleH.build(g, w["leaf"], w["eta"], w["aca_eps"], w["lattice"], lattice_rows=rows_sel)
    build_s = time.perf_counter() - t0
    lat_rows = H.lattice_row_ranges(rows_sel)
    nrows = sum(e - s for s, e in lat_rows)
    scale = f.n / nrows
    forms = {}
    with threadpool_limits(limits=threads):
        per, reps, el, y = _timed(lambda: H.matvec(x), 10.0)
    forms["block_loop_all_threads"] = dict(matvec_per_s=1.0 / (per * scale), threads=threads, reps=reps, s=el)
    with threadpool_limits(limits=1):
        per, reps, el, _ = _timed(lambda: H.matvec(x), 10.0)
    forms["block_loop_1_thread"] = dict(matvec_per_s=1.0 / (per * scale), threads=1, reps=reps, s=el)
    for th in (1, threads):
        S = SparseHMatrix(H, threads=th)
        with threadpool_limits(limits=1):
            per, reps, el, _ = _timed(lambda: S.matvec(x), 5.0)
        S.close()
        forms[f"sparse_csr_{'1_thread' if th == 1 else 'all_threads'}"] = dict(
            matvec_per_s=1.0 / (per * scale), threads=th, reps=reps, s=el)
    per, reps, el, _ = _timed(lambda: fft_grid_product(f.nx, f.ny, f.h, f.slip, MU, NU, x), 5.0)
    forms["exact_fft_full_matrix"] = dict(matvec_per_s=1.0 / per, threads=1, reps=reps, s=el,
                                          note="the dense definition y = A x, whole matrix, no row sampling")
    # oracle Runge-Kutta steps on the 2048-element fault (its own H-matrix)
    w0 = WORKLOADS["planar64x32"]
    f0 = config_fault("planar64x32")
    p0 = friction_params(f0)
    g0 = CoplanarRectGeometry(f0.verts, f0.slip_dir, MU, NU)
    with threadpool_limits(limits=threads):
        H0 = OracleH.build(g0, w0["leaf"], w0["eta"], w0["aca_eps"], w0["lattice"])
        y0 = fr.initial_state(10.0 ** (-12.0 + 3.0 * np.random.default_rng(0).random(f0.n)), p0, p0["sigma"])
        t0 = time.perf_counter()
        run = ork.integrate(lambda z: fr.rhs(z, p0, H0.matvec), y0, 1.0, 60)
        el = time.perf_counter() - t0
    forms["rk45_planar64x32"] = dict(steps_per_s=60 / el, attempts=len(run["log"]), threads=threads, s=el,
                                     note="N = 2048, 60 accepted steps from steady state, block-loop products")
    head = forms["block_loop_all_threads"]
    # compare the oracle's sampled rows with the GPU product on the same rows
    idx = np.concatenate([H.perm[s:e] for s, e in lat_rows])
    err = float(np.linalg.norm(y[idx] - y_gpu[idx]) / np.linalg.norm(y[idx]))
    cpu = open("/proc/cpuinfo").read()
    model = next((l.split(":", 1)[1].strip() for l in cpu.splitlines() if l.startswith("model name")), "unknown")
    log("[bench] cpu baseline: " + ", ".join(
        f"{k} {v.get('matvec_per_s', v.get('steps_per_s')):.2f}" for k, v in forms.items()))
    return {
        "value": head["matvec_per_s"], "unit": "matvec/s", "cores": threads, "kind": "oracle",
        "sample": (f"oracle FP64 H-matrix product (NumPy block loop, BLAS on {threads} threads) over lattice "
                   f"block-rows {list(rows_sel)} = {nrows} of {f.n} rows, {head['reps']} products in "
                   f"{head['s']:.1f} s, scaled by {scale:.1f}; oracle build of the sample {build_s:.1f} s "
                   f"(untimed); the other forms under 'forms'"),
        "forms": forms,
        "cpu_model": model, "host_threads_available": threads,
        "sample_rel_err_gpu_f32_vs_oracle": err,
    }


def _timed_share(torch, hm, rk, p, phi, tau, n_steps, dev):
    """The products' share of the GPU time of the integration, measured in
    the run itself: the same n_steps from the same initial state again,
    with wall-clock stamps around each stage's products and each attempt
    (rs_rk45_run_timed)."""
    n = phi.shape[0]
    rk.state.t, rk.state.dt, rk.state.accepted, rk.state.rejected = 0.0, 1.0, 0, 0
    y = torch.tensor(np.concatenate([phi, tau, p["sigma"]]), device=dev)
    D = torch.zeros(n, dtype=torch.float64, device=dev)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rk.run_timed(y, D, 2, use_graph=True, stream=s)    # capture + warm-up
        rk.state.t, rk.state.dt, rk.state.accepted, rk.state.rejected = 0.0, 1.0, 0, 0
        y.copy_(torch.tensor(np.concatenate([phi, tau, p["sigma"]]), device=dev))
        D.zero_()
        s.synchronize()
        t0 = time.perf_counter()
        tm = rk.run_timed(y, D, n_steps, use_graph=True, stream=s)
        s.synchronize()
        tm["wall_s"] = time.perf_counter() - t0
    tm["note"] = ("device wall-clock stamps before and after each stage's products and around each attempt, "
                  "in a second run of the same steps from the same state; hmvm_share = product_ms / attempt_ms")
    log(f"[bench] measured product share: {tm['product_ms']:.1f} of {tm['attempt_ms']:.1f} ms of GPU time "
        f"({100 * tm['hmvm_share']:.1f} %), {tm['attempts']} attempts")
    return tm


def rk45_run(torch, hm, f, w, x_np, n_steps):
    """Quasi-dynamic rate-and-state simulation on the benchmark fault with the
    FP32 batched product: adaptive RK45 with the step control on the GPU,
    attempts replayed from a HIP graph on a side stream."""
    from paper_2110_12165_amd.tuning import bench_options
    from synth import friction_params
    from synth.faults import MU, NU

    p = friction_params(f)
    dev = torch.device("cuda:0")
    H = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, **bench_options(WORKLOAD, "batched_f32"))
    a, b, dc = (torch.tensor(p[k], device=dev) for k in ("a", "b", "dc"))
    # steady state at the log-uniform slip rates of the product benchmark (eqs. 7-8)
    V = x_np
    phi = p["f0"] + p["b"] * np.log(p["V0"] / V)
    tau = p["a"] * p["sigma"] * np.arcsinh(V / (2 * p["V0"]) * np.exp(phi / p["a"]))
    y = torch.tensor(np.concatenate([phi, tau, p["sigma"]]), device=dev)
    D = torch.zeros(f.n, dtype=torch.float64, device=dev)
    rk = hm.RK45(H, None, a, b, dc, p["V0"], p["f0"], p["eta_rad"], p["V_pl"])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rk.run(y, D, 2, use_graph=True, stream=s)          # capture + warm-up
        s.synchronize()
        t_sim0, acc0, rej0 = rk.t, rk.state.accepted, rk.state.rejected
        t0 = time.perf_counter()
        rk.run(y, D, n_steps, use_graph=True, stream=s)
        s.synchronize()
        wall = time.perf_counter() - t0
    attempts = (rk.state.accepted - acc0) + (rk.state.rejected - rej0)
    t_end, dt_end = rk.t, rk.dt
    share = _timed_share(torch, hm, rk, p, phi, tau, n_steps, dev)
    H.close()
    # FP32 against FP64 factors on the whole run: each with its own step
    # control from the same initial state; the simulated time at which the
    # largest slip rate first reaches 1e-3 m/s (the onset of the first event)
    # and the slip then.  Steps sitting at the explicit stability limit make
    # a replay of one run's steps with the other's factors diverge, so the
    # runs are compared at this physical marker instead.
    onset = {}
    for variant in ("batched_f32", "batched_f64"):
        HH = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, **bench_options(WORKLOAD, variant))
        rr = hm.RK45(HH, None, a, b, dc, p["V0"], p["f0"], p["eta_rad"], p["V_pl"])
        yy = torch.tensor(np.concatenate([phi, tau, p["sigma"]]), device=dev)
        DD = torch.zeros(f.n, dtype=torch.float64, device=dev)
        a_d = a
        hit = None
        for k in range(3 * n_steps):
            rr.run(yy, DD, 1, use_graph=False)
            ph, ta, sg = yy[:f.n], yy[f.n:2 * f.n], yy[2 * f.n:]
            vmax = float(torch.max(2 * p["V0"] * torch.exp(-ph / a_d) * torch.sinh(ta / (a_d * sg))))
            if vmax >= 1e-3:
                hit = (k + 1, rr.t, DD.cpu().numpy())
                break
        HH.close()
        onset[variant] = hit
    ev = {}
    if onset["batched_f32"] and onset["batched_f64"]:
        (k32, t32, d32), (k64, t64, d64) = onset["batched_f32"], onset["batched_f64"]
        ev = {"steps_f32": k32, "steps_f64": k64, "t_f32": t32, "t_f64": t64,
              "t_rel_diff": abs(t32 - t64) / t64,
              "slip_rel_diff": float(np.max(np.abs(d32 - d64)) / np.max(np.abs(d64)))}
        log(f"[bench] rk45 onset of the first event (max V >= 1e-3 m/s): FP32 t = {t32:.6e} s after {k32} steps, "
            f"FP64 t = {t64:.6e} s after {k64} steps (relative {ev['t_rel_diff']:.1e}); slip then differs by "
            f"{ev['slip_rel_diff']:.1e} of its largest value")
    log(f"[bench] rk45: {n_steps} steps, {attempts} attempts in {wall:.3f} s, simulated {t_end - t_sim0:.3e} s")
    return {"accepted_steps": n_steps, "attempts": attempts, "wall_s": wall,
            "steps_per_s": n_steps / wall, "attempts_per_s": attempts / wall,
            "simulated_s": t_end - t_sim0, "simulated_s_per_wall_s": (t_end - t_sim0) / wall,
            "hmvm_share": share["hmvm_share"], "hmvm_share_measurement": share, "dt_last": dt_end,
            "event_onset_f32_vs_f64": ev,
            "note": "Cash-Karp RK45, eps_RK 1e-4, graph-replayed attempts; friction a=0.010, b=0.015/0.005, "
                    "d_c=0.01 m, sigma=50 MPa, V_pl=1e-9 m/s; start from steady state at the benchmark slip rates"}


def ensemble(torch, hm, workloads, reps=20):
    """64-member ensemble product on MFMA (hmat_matmat, BF16x6 and BF16x3)
    against 64 single-vector FP32 batched products on the same handle."""
    from paper_2110_12165_amd.tuning import bench_options
    from synth import TRIANGLE_WORKLOADS, WORKLOADS, config_fault, config_triangle_fault, loguniform_rates
    from synth.faults import MU, NU

    out = {}
    dev = torch.device("cuda:0")
    for name in workloads:
        tri = name in TRIANGLE_WORKLOADS
        w = (TRIANGLE_WORKLOADS if tri else WORKLOADS)[name]
        f = (config_triangle_fault if tri else config_fault)(name)
        opts = bench_options(name, "batched_f32") if name in ("dip30_480x256",) else dict(
            aca_eps=w["aca_eps"], eta=w["eta"], leaf=w["leaf"], lattice=w["lattice"], prec="f32",
            kernel="split", build_device=1)
        H = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, max_nrhs=64, **opts)
        info = H.info()
        X = torch.tensor(loguniform_rates(f.n, 3, nrhs=64), device=dev)
        Y = torch.empty_like(X)
        cols = [X[:, c].contiguous() for c in range(64)]
        yv = torch.empty(f.n, dtype=torch.float64, device=dev)

        def timed(fn):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        ms_x6 = timed(lambda: H.matmat(X, Y=Y, mode="x6"))
        ms_x3 = timed(lambda: H.matmat(X, Y=Y, mode="x3"))
        ms_vec = timed(lambda: [H.matvec(c, y=yv) for c in cols])
        Y6 = H.matmat(X, mode="x6").cpu().numpy()
        Y3 = H.matmat(X, mode="x3").cpu().numpy()
        Yv = np.stack([H.matvec(c).cpu().numpy() for c in cols], axis=1)
        entries = info["dense_entries"] + info["lr_entries"]
        H.close()
        torch.cuda.empty_cache()
        r6 = float(np.linalg.norm(Y6 - Yv) / np.linalg.norm(Yv))
        r3 = float(np.linalg.norm(Y3 - Yv) / np.linalg.norm(Yv))
        res = {"N": f.n, "members": 64, "matrix": "A (shear)", "factor_bytes": info["factor_bytes"],
               "wave_groups": info["mm_groups"],
               "ms_mfma_bf16x6": ms_x6, "ms_mfma_bf16x3": ms_x3, "ms_64_fp32_matvecs": ms_vec,
               "speedup_x6_vs_64_matvecs": ms_vec / ms_x6, "speedup_x3_vs_64_matvecs": ms_vec / ms_x3,
               "member_products_per_s_x6": 64e3 / ms_x6,
               "mfma_tflops_x6": 6 * 2 * entries * 64 / (ms_x6 * 1e-3) / 1e12,
               "mfma_util_x6": 6 * 2 * entries * 64 / (ms_x6 * 1e-3) / 2.5e15,
               "factor_gbs_x6": info["factor_bytes"] / (ms_x6 * 1e-3) / 1e9,
               "rel_diff_x6_vs_fp32_matvecs": r6, "rel_diff_x3_vs_fp32_matvecs": r3}
        log(f"[bench] ensemble {name}: x6 {ms_x6:.3f} ms, x3 {ms_x3:.3f} ms, 64 matvecs {ms_vec:.3f} ms "
            f"(x{ms_vec / ms_x6:.1f}), rel x6 {r6:.1e} x3 {r3:.1e}")
        out[name] = res
    return out


def ensemble_rk(torch, hm, n_steps, members=64, mode="x3", n_single=4, name="thrust_150x70"):
    """64 rate-and-state simulations on one N = 21000 fault advanced together
    (rs_ens_rk45_run: per-member FP64 state and step control, one BF16x3 MFMA
    ensemble product per matrix and stage), against single simulations with
    the FP32 single-vector products (rs_rk45_run), n_single of them timed and
    the time scaled to all members.  On the curved thrust fault (triangles)
    the normal stress evolves too: products with A and B."""
    from synth import TRIANGLE_WORKLOADS, WORKLOADS, config_fault, config_triangle_fault, ensemble_params
    from synth.faults import MU, NU

    tri = name in TRIANGLE_WORKLOADS
    w = (TRIANGLE_WORKLOADS if tri else WORKLOADS)[name]
    f = (config_triangle_fault if tri else config_fault)(name)
    n = f.n
    dev = torch.device("cuda:0")
    opts = dict(aca_eps=w["aca_eps"], eta=w["eta"], leaf=w["leaf"], lattice=w["lattice"], prec="f32",
                kernel="split", max_nrhs=64, build_device=1, transpose=0)
    H = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, component=0, **opts)
    HB = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, component=1, **opts) if tri else None
    p = ensemble_params(f, members, 3)
    V = 10.0 ** (-12.0 + 3.0 * np.random.default_rng(5).random((n, members)))
    phi = p["f0"] + p["b"] * np.log(p["V0"] / V)
    tau = p["a"] * p["sigma"][:, None] * np.arcsinh(V / (2 * p["V0"]) * np.exp(phi / p["a"]))
    phi = phi + np.random.default_rng(105).uniform(-0.05, 0.05, (n, members))
    y0 = np.stack([phi, tau, np.repeat(p["sigma"][:, None], members, 1)])
    a, b, dc = (torch.tensor(np.ascontiguousarray(p[k]), device=dev) for k in ("a", "b", "dc"))
    consts = (p["V0"], p["f0"], p["eta_rad"], p["V_pl"])
    s = torch.cuda.Stream()
    ens = hm.EnsembleRK45(H, HB, a, b, dc, *consts, mode=mode)
    y = torch.tensor(y0, device=dev)
    D = torch.zeros((n, members), dtype=torch.float64, device=dev)
    with torch.cuda.stream(s):
        ens.run(y, D, 2, use_graph=True, stream=s)
        s.synchronize()
        acc0, rej0 = ens.accepted.copy(), ens.rejected.copy()
        t0 = time.perf_counter()
        ens.run(y, D, n_steps, use_graph=True, stream=s)
        s.synchronize()
        wall = time.perf_counter() - t0
    attempts = int(np.max((ens.accepted - acc0) + (ens.rejected - rej0)))
    # single simulations of the first n_single members, same steps
    single = 0.0
    single_attempts = 0
    for r in range(n_single):
        ar, br, dcr = (t[:, r].contiguous() for t in (a, b, dc))
        rk = hm.RK45(H, HB, ar, br, dcr, *consts)
        yr = torch.tensor(np.ascontiguousarray(y0[:, :, r].reshape(-1)), device=dev)
        Dr = torch.zeros(n, dtype=torch.float64, device=dev)
        with torch.cuda.stream(s):
            rk.run(yr, Dr, 2, use_graph=True, stream=s)
            s.synchronize()
            a0 = rk.state.accepted + rk.state.rejected
            t1 = time.perf_counter()
            rk.run(yr, Dr, n_steps, use_graph=True, stream=s)
            s.synchronize()
            single += time.perf_counter() - t1
        single_attempts += rk.state.accepted + rk.state.rejected - a0
    single_all = single / n_single * members
    sig_moved = float((y[2] - torch.tensor(y0[2], device=dev)).abs().max())
    H.close()
    if HB is not None:
        HB.close()
    torch.cuda.empty_cache()
    log(f"[bench] ensemble rk45 {name} ({'A and B' if tri else 'A'}): {members} members x {n_steps} steps in "
        f"{wall:.3f} s ({attempts} attempts); "
        f"single simulations {single / n_single:.3f} s each -> {single_all:.3f} s for {members} (x{single_all / wall:.1f})")
    return {"workload": name, "N": n, "matrices": "A and B" if tri else "A", "members": members, "mode": mode,
            "steps_per_member": n_steps,
            "attempts": attempts, "wall_s": wall, "member_steps_per_s": members * n_steps / wall,
            "single_wall_s_each": single / n_single, "single_attempts_mean": single_attempts / n_single,
            "speedup_vs_single_runs": single_all / wall, "sigma_change_max_pa": sig_moved,
            "note": "per-element a - b ~ U[-0.006, 0.004] (b = 0.015), d_c log-uniform [0.005, 0.05] m (seed 3); "
                    + ("sigma 20-120 MPa rising with depth; " if tri else "sigma 50 MPa; ")
                    + "graph-replayed attempts; single runs use the FP32 single-vector products"}


def nonplanar(torch, hm, reps=50, rk_steps=500):
    """Curved thrust fault of 21000 triangles (dip 30 +/- 10 degrees down dip):
    shear (A) and normal (B) matrices, FP32-batched against FP64-plain."""
    from synth import TRIANGLE_WORKLOADS, config_triangle_fault, loguniform_rates
    from synth.faults import MU, NU

    name = "thrust_150x70"
    w = TRIANGLE_WORKLOADS[name]
    f = config_triangle_fault(name)
    dev = torch.device("cuda:0")
    x = torch.tensor(loguniform_rates(f.n, w["seed"]), device=dev)
    y = torch.empty_like(x)
    out = {"workload": name, "N": f.n}

    def timed(H):
        for _ in range(5):
            H.matvec(x, y=y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            H.matvec(x, y=y)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    for comp, label in ((0, "A"), (1, "B")):
        res = {}
        ys = {}
        for prec, kernel in (("f32", "split"), ("f64", "plain")):
            t0 = time.perf_counter()
            H = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, component=comp, aca_eps=w["aca_eps"], eta=w["eta"],
                                 leaf=w["leaf"], lattice=w["lattice"], prec=prec, kernel=kernel)
            build = time.perf_counter() - t0
            info = H.info()
            ms = timed(H)
            ys[prec] = H.matvec(x).cpu().numpy()
            H.close()
            res[f"{prec}_{kernel}"] = {"ms": ms, "matvec_per_s": 1e3 / ms, "build_s": build,
                                       "factor_bytes": info["factor_bytes"],
                                       "gbs": info["alg_bytes"] / (ms * 1e-3) / 1e9}
        # the same FP32 matrix constructed on the device
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, component=comp, aca_eps=w["aca_eps"], eta=w["eta"],
                             leaf=w["leaf"], lattice=w["lattice"], prec="f32", kernel="split", build_device=1)
        torch.cuda.synchronize()
        res["f32_split"]["build_device_s"] = time.perf_counter() - t0
        yd = H.matvec(x).cpu().numpy()
        H.close()
        res["rel_diff_device_vs_host_build"] = float(np.linalg.norm(yd - ys["f32"]) / np.linalg.norm(ys["f32"]))
        res["n_lr"], res["n_dense"] = info["n_lr"], info["n_dense"]
        res["stored_fraction"] = (info["dense_entries"] + info["lr_entries"]) / float(f.n) ** 2
        res["speedup_f32_batched_vs_f64_plain"] = res["f64_plain"]["ms"] / res["f32_split"]["ms"]
        res["rel_diff_f32_vs_f64"] = float(np.linalg.norm(ys["f32"] - ys["f64"]) / np.linalg.norm(ys["f64"]))
        out[label] = res
        log(f"[bench] nonplanar {label}: FP32 batched {res['f32_split']['ms'] * 1e3:.1f} us, FP64 plain "
            f"{res['f64_plain']['ms'] * 1e3:.1f} us (x{res['speedup_f32_batched_vs_f64_plain']:.1f}), "
            f"rel {res['rel_diff_f32_vs_f64']:.1e}, stored {100 * res['stored_fraction']:.1f} % of dense, "
            f"build {res['f32_split']['build_s']:.2f} s host, {res['f32_split']['build_device_s']:.2f} s device "
            f"(products differ by {res['rel_diff_device_vs_host_build']:.1e})")
    out["rk45"] = nonplanar_rk(torch, hm, f, w, rk_steps)
    torch.cuda.empty_cache()
    return out


def nonplanar_rk(torch, hm, f, w, n_steps):
    """Rate-and-state run on the nonplanar fault with both products: the
    shear stress through A and the normal stress through B (eqs. 9-12),
    FP32 factors built on the device, graph-replayed attempts, from steady
    state at log-uniform slip rates."""
    from synth import loguniform_rates, triangle_friction_params
    from synth.faults import MU, NU

    p = triangle_friction_params(f)
    dev = torch.device("cuda:0")
    opts = dict(aca_eps=w["aca_eps"], eta=w["eta"], leaf=w["leaf"], lattice=w["lattice"], prec="f32",
                kernel="split", build_device=1, transpose=0)
    HA = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, component=0, **opts)
    HB = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, component=1, **opts)
    a, b, dc = (torch.tensor(p[k], device=dev) for k in ("a", "b", "dc"))
    V = loguniform_rates(f.n, w["seed"])
    phi = p["f0"] + p["b"] * np.log(p["V0"] / V)
    tau = p["a"] * p["sigma"] * np.arcsinh(V / (2 * p["V0"]) * np.exp(phi / p["a"]))
    y = torch.tensor(np.concatenate([phi, tau, p["sigma"]]), device=dev)
    D = torch.zeros(f.n, dtype=torch.float64, device=dev)
    rk = hm.RK45(HA, HB, a, b, dc, p["V0"], p["f0"], p["eta_rad"], p["V_pl"])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rk.run(y, D, 2, use_graph=True, stream=s)          # capture + warm-up
        s.synchronize()
        t_sim0, acc0, rej0 = rk.t, rk.state.accepted, rk.state.rejected
        t0 = time.perf_counter()
        rk.run(y, D, n_steps, use_graph=True, stream=s)
        s.synchronize()
        wall = time.perf_counter() - t0
    attempts = (rk.state.accepted - acc0) + (rk.state.rejected - rej0)
    sig = y[2 * f.n:].cpu().numpy()
    t_end, dt_end = rk.t, rk.dt
    share = _timed_share(torch, hm, rk, p, phi, tau, n_steps, dev)
    HA.close()
    HB.close()
    out = {"accepted_steps": n_steps, "attempts": attempts, "wall_s": wall, "steps_per_s": n_steps / wall,
           "simulated_s": t_end - t_sim0, "simulated_s_per_wall_s": (t_end - t_sim0) / wall, "dt_last": dt_end,
           "sigma_change_max_pa": float(np.max(np.abs(sig - p["sigma"]))),
           "hmvm_share": share["hmvm_share"], "hmvm_share_measurement": share}
    log(f"[bench] nonplanar rk45 (A and B): {n_steps} steps, {attempts} attempts in {wall:.3f} s, simulated "
        f"{out['simulated_s']:.3e} s; normal stress moved by up to {out['sigma_change_max_pa']:.3e} Pa")
    return out


def autotune(torch, hm, f, w, x, steps, warmup):
    """hmat_autotune on the benchmark matrix: it times the plain product and
    every batched schedule (waves per workgroup of both phases, split or
    persistent launch) on the handle's own blocks and keeps the fastest;
    reports its pick and the product rate with it."""
    from synth.faults import MU, NU
    H = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, aca_eps=w["aca_eps"], eta=w["eta"], leaf=w["leaf"],
                         lattice=w["lattice"], prec="f32", kernel="auto", transpose=0, build_device=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = H.autotune(reps=10)
    tune_s = time.perf_counter() - t0
    y = torch.empty_like(x)
    ms, _, _ = time_products(torch, H, x, y, steps, warmup)
    H.close()
    torch.cuda.empty_cache()
    out = {"picked": {"kernel": info["kernel"], "wg_waves": info["wg_waves"], "wg_waves_p1": info["wg_waves_p1"]},
           "autotune_s": tune_s, "matvec_per_s": 1e3 / ms, "ms": ms}
    log(f"[bench] autotune: picked {info['kernel']} {info['wg_waves']}/{info['wg_waves_p1']} waves in {tune_s:.1f} s; "
        f"{1e3 / ms:.1f} matvec/s with it")
    return out


def construction(torch, hm, f, opts, x):
    """Build time of the headline matrix (FP32 batched, with the transposed
    layout) from the element geometry: host ACA on all host threads versus
    ACA and dense entries on the GPU.  Both include packing and upload; the
    block lists must agree (same ranks), the products to FP32 rounding."""
    from synth.faults import MU, NU
    out = {}
    ys = {}
    for dev_build in (0, 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, build_device=dev_build, **opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        info = H.info()
        ys[dev_build] = H.matvec(x).cpu().numpy()
        out["device_s" if dev_build else "host_s"] = dt
        out["n_lr_device" if dev_build else "n_lr_host"] = info["n_lr"]
        out["sum_rank_device" if dev_build else "sum_rank_host"] = info["sum_rank"]
        H.close()
        torch.cuda.empty_cache()
    out["rel_diff_products"] = float(np.linalg.norm(ys[1] - ys[0]) / np.linalg.norm(ys[0]))
    out["host_threads"] = len(os.sched_getaffinity(0))
    log(f"[bench] construction: host {out['host_s']:.2f} s, device {out['device_s']:.2f} s; ranks "
        f"{out['sum_rank_host']} / {out['sum_rank_device']}; products differ by {out['rel_diff_products']:.1e}")
    return out


def sweeps(torch, hm, steps=50, warmup=5):
    """Stored entries, build time and FP32 product time of the benchmark
    fault against N (four sizes, lattice 32) and against the lattice size at
    N = 122880 (lattice 1: the normal H-matrix).  Device construction,
    no transposed layout."""
    from synth import LATTICE_SWEEP, SIZE_SWEEP, WORKLOADS, config_fault, loguniform_rates
    from synth.faults import MU, NU
    dev = torch.device("cuda:0")

    def one(name, lattice):
        w = WORKLOADS[name]
        f = config_fault(name)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, aca_eps=w["aca_eps"], eta=w["eta"], leaf=w["leaf"],
                             lattice=lattice, prec="f32", kernel="split", transpose=0, build_device=1)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        info = H.info()
        x = torch.tensor(loguniform_rates(f.n, w["seed"]), device=dev)
        y = torch.empty_like(x)
        ms, _, _ = time_products(torch, H, x, y, steps, warmup)
        H.close()
        torch.cuda.empty_cache()
        entries = info["dense_entries"] + info["lr_entries"]
        r = dict(workload=name, N=f.n, lattice=lattice, build_s=build_s, stored_frac=entries / float(f.n) ** 2,
                 factor_gb=info["factor_bytes"] / 1e9, n_lr=info["n_lr"], n_dense=info["n_dense"],
                 max_rank=info["max_rank"], us_per_product=ms * 1e3,
                 gbs=info["alg_bytes"] / (ms * 1e-3) / 1e9)
        log(f"[bench] sweep {name} lattice {lattice}: N={f.n}, stored {100 * r['stored_frac']:.2f} %, "
            f"{r['factor_gb']:.3f} GB, build {build_s:.2f} s, {r['us_per_product']:.1f} us/product "
            f"({r['gbs']:.0f} GB/s)")
        return r

    out = {"size": [one(name, WORKLOADS[name]["lattice"]) for name in SIZE_SWEEP]}
    out["lattice"] = [one("dip30_480x256", L) for L in LATTICE_SWEEP]
    return out


def adjoint_run(torch, hm, n_steps, ckpt_every=50, name="thrust_150x70"):
    """Gradient of the final-slip misfit L = 1/2 |D_M - D_target|^2 for
    per-element a (b fixed) and d_c on an N = 21000 fault with FP32 factors:
    a controlled run logs its n_steps accepted steps; the target slip comes
    from a perturbed by U(-1e-3, 1e-3) (seed 4), integrated with its own step
    control to the same final time; then the timed part: the frozen-step
    replay writing checkpoints every ckpt_every steps, and the adjoint sweep
    (segments recomputed from their checkpoints, one transposed product per
    matrix and stage).  On the curved thrust fault (triangles) both A and B
    enter (shear and normal stress)."""
    from synth import (TRIANGLE_WORKLOADS, WORKLOADS, config_fault, config_triangle_fault, friction_params,
                       triangle_friction_params)
    from synth.faults import MU, NU

    tri = name in TRIANGLE_WORKLOADS
    w = (TRIANGLE_WORKLOADS if tri else WORKLOADS)[name]
    f = (config_triangle_fault if tri else config_fault)(name)
    p = (triangle_friction_params if tri else friction_params)(f)
    n = f.n
    dev = torch.device("cuda:0")
    opts = dict(aca_eps=w["aca_eps"], eta=w["eta"], leaf=w["leaf"], lattice=w["lattice"], prec="f32",
                kernel="split", build_device=1)
    H = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, component=0, **opts)
    HB = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, component=1, **opts) if tri else None
    mats = [H] + ([HB] if tri else [])
    a, b, dc = (torch.tensor(p[k], device=dev) for k in ("a", "b", "dc"))
    # steady state at log-uniform slip rates (seed 3), then the state variable kicked by U(-0.05, 0.05)
    V = 10.0 ** (-12.0 + 3.0 * np.random.default_rng(3).random(n))
    phi = p["f0"] + p["b"] * np.log(p["V0"] / V)
    tau = p["a"] * p["sigma"] * np.arcsinh(V / (2 * p["V0"]) * np.exp(phi / p["a"]))
    phi = phi + np.random.default_rng(103).uniform(-0.05, 0.05, n)
    y0 = np.concatenate([phi, tau, p["sigma"]])
    consts = (p["V0"], p["f0"], p["eta_rad"], p["V_pl"])
    rk = hm.RK45(H, HB, a, b, dc, *consts)
    y = torch.tensor(y0, device=dev)
    D = torch.zeros(n, dtype=torch.float64, device=dev)
    log_dt = torch.zeros(n_steps, dtype=torch.float64, device=dev)
    rk.run(y, D, n_steps, use_graph=False, dt_log=log_dt)
    dts = log_dt.cpu().numpy()
    T = rk.t
    at = a + torch.tensor(np.random.default_rng(4).uniform(-1e-3, 1e-3, n), device=dev)
    rkt = hm.RK45(H, HB, at, b, dc, *consts)
    yt = torch.tensor(y0, device=dev)
    D_t = torch.zeros(n, dtype=torch.float64, device=dev)
    while rkt.t + rkt.dt < T:
        rkt.step(yt, D_t)
    rkt.dt = T - rkt.t
    rkt.attempt(yt, D_t, force=1)
    # warm-up of the timed calls (also sizes the adjoint workspace)
    yw = torch.tensor(y0, device=dev)
    ck = rk.replay(yw, None, dts[:ckpt_every], ckpt_every=ckpt_every)
    rk.adjoint(ck, dts[:ckpt_every], ckpt_every, torch.zeros_like(yw))
    torch.cuda.synchronize()
    y = torch.tensor(y0, device=dev)
    D = torch.zeros(n, dtype=torch.float64, device=dev)
    t0 = time.perf_counter()
    ckpt = rk.replay(y, D, dts, ckpt_every=ckpt_every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    Dbar = D - D_t
    ybar = torch.zeros_like(y)
    _, ga, gdc = rk.adjoint(ckpt, dts, ckpt_every, ybar, Dbar)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    x = torch.tensor(V, device=dev)
    yv = torch.empty_like(x)
    ms_f, ms_t = 0.0, 0.0   # one product with each matrix, and with each transpose
    for M in mats:
        ms_f += M.profile(x, yv, reps=20)["ms_product"]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(3):
            M.matvec_T(x, y=yv)
        e0.record()
        for _ in range(20):
            M.matvec_T(x, y=yv)
        e1.record()
        torch.cuda.synchronize()
        ms_t += e0.elapsed_time(e1) / 20
    fwd, bwd = t1 - t0, t2 - t1
    prod_s = (12 * n_steps * ms_f + 6 * n_steps * ms_t) * 1e-3
    for M in mats:
        M.close()
    torch.cuda.empty_cache()
    loss = 0.5 * float((Dbar * Dbar).sum())
    log(f"[bench] adjoint {name} ({'A and B' if tri else 'A'}): N={n}, {n_steps} steps to t={T:.3e} s, "
        f"forward {fwd:.3f} s, adjoint {bwd:.3f} s, L={loss:.3e}")
    return {"workload": name, "N": n, "matrices": "A and B" if tri else "A", "steps": n_steps,
            "ckpt_every": ckpt_every, "factor_storage": "f32",
            "simulated_s": T, "forward_replay_s": fwd, "adjoint_s": bwd, "gradient_s": fwd + bwd,
            "products": 18 * n_steps * len(mats), "ms_products": ms_f, "ms_products_T": ms_t,
            "hmvm_share": prod_s / (fwd + bwd), "loss": loss,
            "grad_a_norm": float(ga.norm()), "grad_dc_norm": float(gdc.norm()),
            "note": "L = 1/2 |D_M - D_target|^2; D_target from a + U(-1e-3, 1e-3) (seed 4) by its own step control "
                    "to the same final time; gradient by the discrete adjoint of the frozen-step replay; "
                    "products per matrix: 6 per step forward, 6 per step recomputed from checkpoints, 6 transposed; "
                    "ms_products(_T): one product with each matrix (its transpose), summed"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants", default="batched_f32,plain_f64,batched_f64")
    ap.add_argument("--rk-steps", type=int, default=1000,
                    help="accepted RK45 steps of the rate-and-state simulation on the same fault (0: skip)")
    ap.add_argument("--ensemble", default="thrust_150x70,dip30_480x256",
                    help="workloads of the 64-member MFMA ensemble product ('' to skip)")
    ap.add_argument("--no-nonplanar", action="store_true", help="skip the triangle-mesh section")
    ap.add_argument("--no-construction", action="store_true", help="skip the host/device build timing")
    ap.add_argument("--no-sweeps", action="store_true", help="skip the size and lattice sweeps")
    ap.add_argument("--no-autotune", action="store_true", help="skip the autotuner run")
    ap.add_argument("--ens-rk-steps", type=int, default=100,
                    help="steps per member of the ensemble integration (0: skip)")
    ap.add_argument("--adjoint-steps", type=int, default=500,
                    help="steps of the adjoint section (0: skip)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the product is not sharded across GPUs "
              "(the sharding is described with the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2110_12165_amd as hm
    from paper_2110_12165_amd.tuning import bench_options
    from synth import WORKLOADS, config_fault, loguniform_rates
    from synth.faults import MU, NU

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    w = WORKLOADS[WORKLOAD]
    f = config_fault(WORKLOAD)
    x_np = loguniform_rates(f.n, w["seed"])
    x = torch.tensor(x_np, device=dev)
    if args.calib_copy_mib:
        src_buf = torch.ones(args.calib_copy_mib * (1 << 18), dtype=torch.float32, device=dev)
        dst_buf = torch.empty_like(src_buf)
        dst_buf.copy_(src_buf)
        torch.cuda.synchronize()
        del src_buf, dst_buf
    results = {}
    outputs = {}
    for variant in args.variants.split(","):
        opts = bench_options(WORKLOAD, variant)
        t0 = time.perf_counter()
        H = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, **opts)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        info = H.info()
        y = torch.empty_like(x)
        log(f"[bench] {variant}: built in {build_s:.1f} s; kernel {info['kernel']}, "
            f"{info['factor_bytes'] / 1e9:.3f} GB of factors")
        ms, product_ms, wall_ms = time_products(torch, H, x, y, args.steps, args.warmup)
        outputs[variant] = H.matvec(x).cpu().numpy()
        # per-launch durations from HIP events recorded by the library on this stream
        pr = H.profile(x, y, reps=args.steps)
        dom = int(np.argmax(pr["ms"]))
        launches = [dict(alg_bytes=b, ms=m, achieved_gbs=b / (m * 1e-3) / 1e9)
                    for b, m in zip(pr["alg_bytes"], pr["ms"])]
        achieved = launches[dom]["achieved_gbs"]
        whole = info["alg_bytes"] / (ms * 1e-3) / 1e9
        results[variant] = dict(ms=ms, product_ms=product_ms, wall_ms=wall_ms, matvec_per_s=1e3 / ms,
                                alg_bytes=info["alg_bytes"], achieved_gbs=achieved, dominant_launch=dom,
                                launches=launches, hbm_frac=achieved / HBM_PEAK_GBS,
                                product_gbs=whole, product_hbm_frac=whole / HBM_PEAK_GBS, build_s=build_s, info=info)
        if variant == "batched_f32":
            # the transposed product (hmat_matvec_T) on its own packed copy of the factors
            for _ in range(args.warmup):
                H.matvec_T(x, y=y)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.steps):
                H.matvec_T(x, y=y)
            e1.record()
            torch.cuda.synchronize()
            ms_t = e0.elapsed_time(e1) / args.steps
            results[variant]["transpose"] = dict(ms=ms_t, matvec_per_s=1e3 / ms_t,
                                                 product_gbs=info["alg_bytes"] / (ms_t * 1e-3) / 1e9)
            # four vectors per call: the split schedule reads each stored entry once for all four
            xs = x.repeat(4)
            ys = torch.empty_like(xs)
            stream_ptr = torch.cuda.current_stream().cuda_stream
            for _ in range(args.warmup):
                H.matvec_raw(xs.data_ptr(), ys.data_ptr(), nrhs=4, ld=f.n, stream_ptr=stream_ptr)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.steps):
                H.matvec_raw(xs.data_ptr(), ys.data_ptr(), nrhs=4, ld=f.n, stream_ptr=stream_ptr)
            e1.record()
            torch.cuda.synchronize()
            ms_4 = e0.elapsed_time(e1) / args.steps
            dev4 = float((ys.view(4, f.n) - ys.view(4, f.n)[0]).abs().max() / ys.view(4, f.n)[0].abs().max())
            results[variant]["multi_rhs"] = dict(nrhs=4, ms=ms_4, vectors_per_s=4e3 / ms_4,
                                                 speedup_vs_single=4 * ms / ms_4, columns_max_rel_diff=dev4)
            log(f"[bench] {variant}: 4 vectors per call {ms_4 * 1e3:.1f} us ({4e3 / ms_4:.0f} vectors/s, "
                f"{4 * ms / ms_4:.2f}x four single products)")
            log(f"[bench] {variant}: transposed product {ms_t * 1e3:.1f} us "
                f"({info['alg_bytes'] / (ms_t * 1e-3) / 1e9:.0f} GB/s)")
        log(f"[bench] {variant}: {1e3 / ms:.1f} matvec/s ({ms * 1e3:.1f} us/product, {whole:.0f} GB/s = "
            f"{100 * whole / HBM_PEAK_GBS:.1f}% of HBM over the product); launches "
            + ", ".join(f"{l['ms'] * 1e3:.1f} us {l['achieved_gbs']:.0f} GB/s" for l in launches))
        H.close()
        torch.cuda.empty_cache()

    head = results["batched_f32"]
    info = head["info"]
    line = {
        "metric": METRIC,
        "value": head["matvec_per_s"],
        "unit": "matvec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 storage, f64 accumulate",
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD, "N": f.n,
            "geometry": "planar 30-deg dipping thrust, 480 x 256 squares of 50 m, full-space coplanar kernel",
            "aca_eps": w["aca_eps"], "leaf": w["leaf"], "eta": w["eta"], "lattice": w["lattice"],
            "x": "log-uniform [1e-12, 1e-9] m/s, seed 2",
            "factor_storage": "f32", "accumulate": "f64", "kernel": info["kernel"],
            "wg_waves": info["wg_waves"], "wg_waves_p1": info["wg_waves_p1"],
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": head["achieved_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": head["hbm_frac"],
            "traffic": TRAFFIC.get((info["kernel"], head["dominant_launch"], source_hash())),
            "kernel": DOMINANT_SYMBOL.get((info["kernel"], head["dominant_launch"]), "?"),
            "launch_alg_bytes": head["launches"][head["dominant_launch"]]["alg_bytes"],
            "launch_ms": head["launches"][head["dominant_launch"]]["ms"],
            "launches": head["launches"],
            "product_gbs": head["product_gbs"],
            "product_frac": head["product_hbm_frac"],
        },
        "hmat": {k: info[k] for k in ("n_dense", "n_lr", "dense_entries", "lr_entries", "max_rank", "sum_rank",
                                      "factor_bytes", "alg_bytes", "n_units_p1", "n_units_p2")},
    }
    for v, r in results.items():
        line[v] = {k: r[k] for k in ("matvec_per_s", "ms", "product_gbs", "product_hbm_frac", "achieved_gbs",
                                     "hbm_frac", "build_s")}
        line[v]["kernel"] = r["info"]["kernel"]
        for extra in ("transpose", "multi_rhs"):
            if extra in r:
                line[v][extra] = r[extra]
    if "plain_f64" in results:
        line["speedup_batched_f32_vs_plain_f64"] = head["matvec_per_s"] / results["plain_f64"]["matvec_per_s"]
    if "batched_f64" in outputs:
        ref = outputs["batched_f64"]
        line["rel_diff_f32_vs_f64_gpu"] = float(np.linalg.norm(outputs["batched_f32"] - ref) / np.linalg.norm(ref))
    def section(key, fn, *fargs):
        # one further section; a failure is logged and recorded under its key,
        # and the line (headline measured above) is still printed
        try:
            line[key] = fn(*fargs)
        except Exception as e:  # noqa: BLE001
            log(f"[bench] {key} failed: {type(e).__name__}: {e}")
            line[key] = {"error": f"{type(e).__name__}: {e}"}

    if not args.no_construction:
        section("construction", construction, torch, hm, f, bench_options(WORKLOAD, "batched_f32"), x)
    if not args.no_autotune:
        section("autotune", autotune, torch, hm, f, w, x, args.steps, args.warmup)
    if not args.no_sweeps:
        section("sweeps", sweeps, torch, hm)
    if args.rk_steps > 0:
        section("rk45", rk45_run, torch, hm, f, w, x_np, args.rk_steps)
    if args.ensemble:
        section("ensemble", ensemble, torch, hm, args.ensemble.split(","))
    if not args.no_nonplanar:
        section("nonplanar", nonplanar, torch, hm)
    if args.ens_rk_steps > 0:
        section("ensemble_rk45", ensemble_rk, torch, hm, args.ens_rk_steps)
    if args.adjoint_steps > 0:
        section("adjoint", adjoint_run, torch, hm, args.adjoint_steps)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle sample) ...")
        section("cpu_baseline", cpu_baseline, f, w, x_np, outputs["batched_f32"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
