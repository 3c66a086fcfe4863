"""Benchmark of the two-site DMRG sigma step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--config cas54_36|cas54_36_sz2|cas22_22]
                    [--precision bf16x3|bf16|fp64] [--fp64-steps K64] [--dav-iters I]
                    [--dav-solve 0|1|2|3] [--no-cpu-baseline]

Workload (default): CAS(54,36)-shaped active space (36 orbitals, 54
electrons, 2Sz = 0), bond dimension D = 4096, middle window (17, 18),
synthetic integrals (seed 36) and a converged-like random MPS (seed 1036).
Operators are built once (dmrg_build_ops, untimed); a timed step is one
sigma = H_eff psi on the resident psi in the mixed precision (split-BF16x3
MFMA, block Hamiltonians in FP64) unless --precision says otherwise.  The
JSON line reports algorithmic sigma TFLOP/s; beside it the FP64 sigma of the
same psi (time, relative difference, Rayleigh-quotient difference, its own
roofline), the Ozaki-scheme sigma (FP64 emulated on INT8, the paper's
47-bit setting) with its roofline, the Davidson step time with the mixed
ladder, a Davidson solve to the paper's eigensolver tolerance (residual
1e-6 with FP64 sigma products) with the mixed ladder and residual
refinement (time to solution, FP64 residual and energy; --dav-solve 1 adds
the ladder alone and FP64 alone for the energy difference), the roofline of
the dominant grouped-GEMM kernel from HIP events the library records around
each launch on its stream, and the CPU oracle timed on a bounded sample of
the same contraction on the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CONFIGS = {
    # name: (K, N, 2Sz, D, integral seed, mps seed)
    "cas54_36": (36, 54, 0, 4096, 36, 1036),
    "cas54_36_sz2": (36, 54, 4, 4096, 36, 1036),
    "cas22_22": (22, 22, 0, 1024, 22, 1022),
}
PEAK_TFLOPS = {"fp64": 78.6, "bf16": 2516.6, "bf16x3": 2516.6}
METRIC = "sigma H·ψ TFLOP/s + Davidson step time, CAS(54,36) D=4096, mixed vs FP64"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def profiled_traffic(profile, sources, key, config):
    """HBM bytes per sigma of a grouped-GEMM family from a committed rocprofv3
    summary under profiles/, if it was taken with these sources (the kernel
    and the schedule that builds its launches) and this launch configuration
    (the value of the `key:` line), else None.  Returns (bytes per sigma,
    launches per sigma)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", profile)
    try:
        text = open(path).read()
        h = hashlib.sha256()
        for src in sources:
            h.update(open(src, "rb").read())
        sha = h.hexdigest()
    except OSError:
        return None
    m_sha = re.search(r"sources_sha256:\s*([0-9a-f]+)", text)
    m_cfg = re.search(re.escape(key) + r":\s*(\S+)", text)
    m_tr = re.search(r"traffic_bytes_per_sigma:\s*([0-9.eE+]+)", text)
    m_ln = re.search(r"launches_per_sigma:\s*(\d+)", text)
    if not (m_sha and m_cfg and m_tr and m_ln) or m_sha.group(1) != sha:
        return None
    if m_cfg.group(1) != config:
        return None
    return float(m_tr.group(1)), int(m_ln.group(1))


def cpu_baseline(m, reps=2, seed=0):
    """The oracle's sigma time on this window, from a stratified sample of
    its partition terms.

    The oracle applies each partition term O_L (x) O_R as dense products of
    enlarged-block operators (BlockSparseSigma.apply_matrix).  Its terms fall
    into 13 classes by the quantum-number change of O_L (O_R carries the
    opposite): H_L (x) 1 and 1 (x) H_R, a+_p S_p / a_p S_p^+ and T_m a_m /
    T_m^+ a+_m (change (+-1, +-1)), A_pq P_pq and its conjugate ((+-2, 0),
    (+-2, +-2)), B_pq Q_pq ((0, 0), (0, +-2)).  The oracle cannot build this
    window's operators in bounded time, so each class is timed with the
    oracle's own contraction on the real enlarged sectors of the window and
    random operators filling every block the class allows (the values do not
    change the work), and the time per class is multiplied by the number of
    terms of that class in the window (counted from the spin-orbitals on each
    side).  Returns (modelled seconds per sigma, seconds timed, classes,
    terms).
    """
    from oracle import blocksparse as bs
    rng = np.random.default_rng(seed)
    i = m.window
    K = m.n_orb
    q_tot = (m.n_elec, m.two_sz)
    Lb = bs.Basis([((s[0], s[1]), s[2]) for s in m.bonds[i]])
    Rb = bs.Basis([((q_tot[0] - s[0], q_tot[1] - s[1]), s[2]) for s in m.bonds[i + 2]])
    EL, ER = bs.Enlarged(Lb, "left"), bs.Enlarged(Rb, "right")
    obj = object.__new__(bs.BlockSparseSigma)
    obj.mps, obj.EL, obj.ER, obj.q_tot = m, EL, ER, q_tot
    Psi = obj.to_matrix(m.psi)

    def rand_op(E, dq):
        blocks = {}
        for kc, qc in enumerate(E.qn):
            kr = E.idx.get((qc[0] + dq[0], qc[1] + dq[1]))
            if kr is not None:
                blocks[(kr, kc)] = rng.normal(size=(E.dim[kr], E.dim[kc]))
        return bs.Op(dq, blocks)

    ML, MR = 2 * (i + 1), 2 * (K - i - 1)  # spin-orbitals left / right of the cut
    hl, hr = ML // 2, MR // 2             # per spin
    counts = {(0, 0): 2 * hl * hl, (0, 2): hl * hl, (0, -2): hl * hl,
              (2, 0): hl * hl, (-2, 0): hl * hl,
              (2, 2): hl * (hl - 1) // 2, (2, -2): hl * (hl - 1) // 2,
              (-2, 2): hl * (hl - 1) // 2, (-2, -2): hl * (hl - 1) // 2}
    for d in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
        counts[d] = hl + hr  # a+_p S_p (or conjugate) for p left, T_m a_m for m right
    t_model, t_spent = 0.0, 0.0
    for dq, cnt in counts.items():
        XL = rand_op(EL, dq)
        XR = rand_op(ER, (-dq[0], -dq[1]))
        t0 = time.perf_counter()
        for _ in range(reps):
            obj.apply_matrix(Psi, [(1.0, XL, XR)])
        dt = (time.perf_counter() - t0) / reps
        t_spent += dt * reps
        t_model += dt * cnt
    # the two block Hamiltonians: one-sided products
    HL, HR = rand_op(EL, (0, 0)), rand_op(ER, (0, 0))
    t0 = time.perf_counter()
    obj.apply_matrix(Psi, [(1.0, HL, None), (1.0, None, HR)])
    dt = time.perf_counter() - t0
    t_spent += dt
    t_model += dt
    return t_model, t_spent, len(counts) + 1, sum(counts.values()) + 2


def su2_bench(ctx, steps):
    """The spin-adapted FP64 sigma (dmrg_su2_plan_*) on the CAS(89,102)-shaped
    S = 5/2 workload with 2048 multiplets a side: plan once, one untimed
    call, then `steps` calls timed between device synchronisations."""
    import torch
    from synthetic.su2 import cas89_102_workload
    t0 = time.perf_counter()
    w = cas89_102_workload()
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan = ctx.su2_plan(w["left_sectors"], w["right_sectors"], w["n"], w["two_s"], w["left_ops"],
                        w["right_ops"], w["pairs"])
    t_plan = time.perf_counter() - t0
    try:
        info = plan.info()
        out = torch.empty_like(w["psi"])
        plan.sigma(w["psi"], out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.sigma(w["psi"], out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
    finally:
        plan.close()
    # split-BF16x3 plan of the same workload, against the FP64 result
    plan3 = ctx.su2_plan(w["left_sectors"], w["right_sectors"], w["n"], w["two_s"], w["left_ops"],
                         w["right_ops"], w["pairs"], precision="bf16x3")
    try:
        out3 = torch.empty_like(w["psi"])
        plan3.sigma(w["psi"], out3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan3.sigma(w["psi"], out3)
        torch.cuda.synchronize()
        ms3 = (time.perf_counter() - t0) / steps * 1e3
    finally:
        plan3.close()
    rel3 = float((torch.linalg.norm(out3 - out) / torch.linalg.norm(out)).item())
    flops = info["flops_stage1"] + info["flops_stage2"]
    tflops = flops / (ms * 1e-3) / 1e12
    csrc = os.path.join(ROOT, "paper_2603_28648_amd", "csrc")
    pt = profiled_traffic("k_gemm_f64_su2_cas89_102_D2048.md",
                          [os.path.join(csrc, "kernels.hip"), os.path.join(csrc, "su2.cpp")],
                          "su2_tiles", os.environ.get("DMRG_SU2_TILE", "128x64,128x64"))
    traffic = pt[0] / pt[1] if pt else None  # bytes per launch
    leg = {"workload": "cas89_102 S=5/2: 51|51 orbitals, 2048 multiplets a side, "
                       f"{len(w['pairs'])} operator pairs, random reduced blocks",
           "psi_size": info["psi_size"], "pairs": len(w["pairs"]),
           "operator_gb": (w["left_data"].numel() + w["right_data"].numel()) * 8 / 1e9,
           "chunks": info["n_chunks"], "segments": info["n_segments"],
           "workspace_gb": info["workspace_bytes"] / 1e9, "flops": flops,
           "flops_stages": [info["flops_stage1"], info["flops_stage2"]],
           "gen_s": round(t_gen, 2), "plan_s": round(t_plan, 2), "ms": ms, "tflops": tflops,
           "bf16x3": {"ms": ms3, "tflops": flops / (ms3 * 1e-3) / 1e12, "speedup_vs_fp64": ms / ms3,
                      "sigma_rel_err_vs_fp64": rel3},
           "roofline": {"bound": "mfma", "achieved": tflops, "peak": PEAK_TFLOPS["fp64"],
                        "unit": "TFLOP/s", "frac": tflops / PEAK_TFLOPS["fp64"], "traffic": traffic,
                        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                        "launches_per_step": 2 * info["n_chunks"],
                        "kernel": "k_gemm_f64 (stage-1 and stage-2 launches of every chunk)"}}
    log(f"[bench] su2 sigma (CAS(89,102) S=5/2, {len(w['pairs'])} pairs, {info['n_chunks']} chunks, "
        f"{info['n_segments']} block products): {ms:.1f} ms, {tflops:.1f} TFLOP/s FP64 "
        f"({100 * tflops / PEAK_TFLOPS['fp64']:.1f}% of peak); plan {t_plan:.1f} s, inputs {t_gen:.1f} s; "
        f"split-BF16x3 {ms3:.1f} ms ({ms / ms3:.2f}x), |dsigma|/|sigma| = {rel3:.2e}")
    del w
    torch.cuda.empty_cache()
    return leg


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="cas54_36", choices=sorted(CONFIGS))
    ap.add_argument("--precision", default="bf16x3", choices=["fp64", "bf16", "bf16x3"],
                    help="precision of the timed sigma steps (the mixed path by default)")
    ap.add_argument("--fp64-steps", type=int, default=3,
                    help="FP64 sigma steps timed beside the headline precision (0: skip)")
    ap.add_argument("--bf16-steps", type=int, default=3,
                    help="plain BF16 sigma steps timed beside the headline (0: skip)")
    ap.add_argument("--dav-iters", type=int, default=4,
                    help="Davidson iterations timed with the mixed ladder (0: skip)")
    ap.add_argument("--dav-solve", type=int, default=3,
                    help="1: also solve to residual 1e-6 with the mixed ladder, with the mixed ladder "
                         "and residual refinement, and with FP64 alone (time-to-solution and energy "
                         "differences; minutes at CAS(54,36)); 2: the mixed ladder only; 3: the "
                         "refined ladder only; 0: skip")
    ap.add_argument("--ozaki-steps", type=int, default=2,
                    help="Ozaki-scheme (FP64 emulated on INT8) sigma steps timed beside the headline (0: skip)")
    ap.add_argument("--su2-steps", type=int, default=3,
                    help="spin-adapted (SU(2)) FP64 sigma steps on the CAS(89,102)-shaped S = 5/2 workload "
                         "with 2048 multiplets a side, timed beside the headline (0: skip)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch each sigma kernel by kernel instead of replaying a captured HIP graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=20,
                    help="repeats of each term class in the CPU-oracle sample")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run a plain device-to-device copy of MB megabytes, 3 times "
                         "(reference for the HBM byte counters), then exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each": 8 * n, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sigma "
              "would shard over Hamiltonian terms with one all-reduce of sigma per "
              "Davidson iteration, which this build does not implement.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_28648_amd import Context
    from synthetic import make_integrals, make_mps, mps_arrays, pack_psi

    K, N, tsz, D, iseed, mseed = CONFIGS[args.config]
    i = K // 2 - 1
    t0 = time.time()
    h, eri = make_integrals(K, iseed)
    m = make_mps(K, N, tsz, D, i, mseed)
    log(f"[bench] inputs K={K} N={N} 2Sz={tsz} D={D} window={i} psi={m.psi_size()} "
        f"({time.time() - t0:.1f}s)")
    stream = torch.cuda.Stream()
    ctx = Context(0, stream=stream.cuda_stream)
    t0 = time.time()
    with torch.cuda.stream(stream):
        ctx.build_ops(i, h=h, eri=eri, n_elec=N, two_sz=tsz, mps_arrays=mps_arrays(m))
    stream.synchronize()
    t_build = time.time() - t0
    info = ctx.sigma_info(args.precision)
    log(f"[bench] build_ops {t_build:.1f}s, {info['n_pairs']} pairs, "
        f"{info['operator_bytes'] / 1e9:.1f} GB operators, {info['flops']:.3e} flop/sigma")
    psi = torch.from_numpy(pack_psi(m.bonds, i, m.psi)).to("cuda")
    psi /= torch.linalg.norm(psi)
    out = torch.empty_like(psi)
    ref = torch.empty_like(psi)
    torch.cuda.synchronize()

    def kernel_roofline(kt, kname, peak, unit, hw_per_flop):
        """Achieved rate of the main-stage grouped-GEMM launches of the timed
        calls: algorithmic FLOPs per launch (times hw_per_flop hardware
        operations per FLOP) over the average launch time from the library's
        HIP events on its stream."""
        n = kt["launches_stage1"] + kt["launches_stage2"]
        ms_k = (kt["ms_stage1"] + kt["ms_stage2"]) / max(1, n)
        fl = (kt["flops_stage1"] + kt["flops_stage2"]) * kt["calls"] / max(1, n)
        ach = hw_per_flop * fl / (ms_k * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
                "kernel": kname, "launches_per_step": n / max(1, kt["calls"]), "avg_launch_ms": ms_k}

    def timed_sigma(prec, steps, warmup, target, kernel_timing):
        """Event times of `steps` sigma calls on the library stream; with
        kernel_timing, also the library's per-launch kernel times over the same
        calls (launched one by one: the timing hook bypasses the graphs)."""
        with torch.cuda.stream(stream):
            for _ in range(warmup):
                ctx.sigma(psi, target, prec)
        stream.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        if kernel_timing:
            ctx.sigma_timing(1)
        tw = time.perf_counter()
        with torch.cuda.stream(stream):
            for k in range(steps):
                ev[k][0].record(stream)
                ctx.sigma(psi, target, prec)
                ev[k][1].record(stream)
        stream.synchronize()
        tw = time.perf_counter() - tw
        kt = ctx.sigma_timing(0) if kernel_timing else None
        times = np.array([a.elapsed_time(b) for a, b in ev])
        return times, kt, tw

    # FP64 reference sigma (also the comparison the metric asks for)
    fp64 = None
    with torch.cuda.stream(stream):
        ctx.sigma(psi, ref, "fp64")
    stream.synchronize()
    ctx.sigma_graphs(not args.no_graphs)
    if args.fp64_steps > 0 and args.precision != "fp64":
        t64, kt64, _ = timed_sigma("fp64", args.fp64_steps, 0, ref, True)
        fp64 = {"ms": float(np.median(t64)), "tflops": info["flops"] / (np.median(t64) * 1e-3) / 1e12}
        fp64["frac_of_fp64_peak"] = fp64["tflops"] / PEAK_TFLOPS["fp64"]
        fp64["roofline"] = kernel_roofline(kt64, "k_gemm_f64_lds", PEAK_TFLOPS["fp64"], "TFLOP/s", 1.0)
        # HBM bytes per launch from the committed FP64 profile (default tiles,
        # direct-to-LDS kernel, same kernel and schedule sources), else None
        fp64["roofline"]["traffic"] = None
        if args.config == "cas54_36" and os.environ.get("DMRG_F64_LDS", "1") != "0":
            csrc = os.path.join(ROOT, "paper_2603_28648_amd", "csrc")
            pt = profiled_traffic("k_gemm_f64_sigma_cas54_36_D4096.md",
                                  [os.path.join(csrc, "kernels.hip"), os.path.join(csrc, "engine.cpp")],
                                  "fp64_tiles", os.environ.get("DMRG_F64_TILE", "128,128x64"))
            if pt is not None:
                fp64["roofline"]["traffic"] = pt[0] / pt[1]
        log(f"[bench] sigma fp64: median {fp64['ms']:.2f} ms ({fp64['tflops']:.2f} TFLOP/s); "
            f"k_gemm_f64_lds {fp64['roofline']['achieved']:.1f} TFLOP/s per launch")
    times, _, t_wall = timed_sigma(args.precision, args.steps, args.warmup, out, False)
    ms = float(np.median(times))
    # per-kernel times for the roofline: a few more steps with the timing hook
    _, kt, _ = timed_sigma(args.precision, min(args.steps, 3), 0, out, True)
    info2 = ctx.sigma_info(args.precision)  # after the first mixed sigma: autotuned launch configuration
    tuned = {"stage1": info2["bf_config_stage1"], "stage2": info2["bf_config_stage2"],
             "tune_ms": info2["tune_ms"]}
    if args.precision != "fp64":
        log(f"[bench] BF16 launch configuration (shape + 16*grouping + 256*segment order): "
            f"stage 1 {tuned['stage1']}, stage 2 {tuned['stage2']}, autotuned in {tuned['tune_ms']:.0f} ms")
    e_ref = float(torch.dot(psi, ref).item())
    e_mix = float(torch.dot(psi, out).item())
    rel = float((torch.linalg.norm(out - ref) / torch.linalg.norm(ref)).item())
    log(f"[bench] sigma {args.precision}: median {ms:.2f} ms, min {times.min():.2f}, "
        f"max {times.max():.2f}; <psi|H|psi> = {e_mix:.10f} (FP64 {e_ref:.10f}); "
        f"|dsigma|/|sigma| = {rel:.2e}")
    tflops = info["flops"] / (ms * 1e-3) / 1e12
    # dominant kernel: the grouped GEMM of the main stages (stage 1 + stage 2)
    n_launch = kt["launches_stage1"] + kt["launches_stage2"]
    ms_kernel = (kt["ms_stage1"] + kt["ms_stage2"]) / max(1, n_launch)
    flops_launch = (kt["flops_stage1"] + kt["flops_stage2"]) * kt["calls"] / max(1, n_launch)
    achieved = flops_launch / (ms_kernel * 1e-3) / 1e12
    kname = "k_gemm_f64_lds" if args.precision == "fp64" else "k_gemm_bf16"
    log(f"[bench] {kname}: {n_launch} launches, avg {ms_kernel:.3f} ms, stage1 "
        f"{kt['ms_stage1'] / kt['calls']:.1f} ms + stage2 {kt['ms_stage2'] / kt['calls']:.1f} ms + "
        f"pinned FP64 {kt['ms_pinned'] / kt['calls']:.1f} ms per sigma; {achieved:.1f} TFLOP/s")
    # plain BF16 sigma (the first rung of the ladder)
    bf16 = None
    if args.bf16_steps > 0 and args.precision != "bf16":
        sb = torch.empty_like(psi)
        tb, _, _ = timed_sigma("bf16", args.bf16_steps, 1, sb, False)
        rel_b = float((torch.linalg.norm(sb - ref) / torch.linalg.norm(ref)).item())
        bf16 = {"ms": float(np.median(tb)), "tflops": info["flops"] / (np.median(tb) * 1e-3) / 1e12,
                "sigma_rel_err_vs_fp64": rel_b}
        bf16["frac_of_bf16_peak"] = bf16["tflops"] / PEAK_TFLOPS["bf16"]
        log(f"[bench] sigma bf16: median {bf16['ms']:.2f} ms ({bf16['tflops']:.1f} TFLOP/s, "
            f"{100 * bf16['frac_of_bf16_peak']:.1f}% of the BF16 peak); |dsigma|/|sigma| = {rel_b:.2e}")
    # Davidson step time with the mixed ladder (FP64 vectors and subspace)
    dav = None
    if args.dav_iters > 0:
        x = psi.clone()
        with torch.cuda.stream(stream):
            r = ctx.davidson(x, tol=1e-12, max_iter=args.dav_iters,
                             ladder=((args.precision, 1e-12), ("fp64", None)))
        stream.synchronize()
        n_sig = sum(r["n_sigma"].values())
        other = (r["time_ms"] - r["sigma_ms"]) / max(1, n_sig)
        dav = {"iterations": r["iterations"], "time_ms": r["time_ms"], "sigma_calls": r["n_sigma"],
               "step_ms": ms + other, "non_sigma_ms_per_step": other, "energy": r["energy"],
               "residual": r["residual"]}
        log(f"[bench] davidson {r['iterations']} iterations: {r['time_ms']:.0f} ms total, "
            f"{other:.2f} ms non-sigma per step -> step {ms + other:.1f} ms")
    # time to solution: the mixed ladder against FP64 alone, same start, residual 1e-6
    solve = None
    if args.dav_solve:
        ladder = (("bf16", 1e-2), ("bf16x3", 1e-4), ("fp64", None))
        res = {}
        runs = (("mixed", ladder, False), ("refined", ladder, True), ("fp64", (("fp64", None),), False))
        runs = {1: runs, 2: runs[:1], 3: runs[1:2]}[args.dav_solve]
        for name, lad, refine in runs:
            x = psi.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with torch.cuda.stream(stream):
                r = ctx.davidson(x, tol=1e-6, max_iter=400, ladder=lad, refine=refine)
            stream.synchronize()
            res[name] = {"time_s": time.perf_counter() - t0, "iterations": r["iterations"],
                         "sigma_calls": r["n_sigma"], "energy": r["energy"], "residual": r["residual"],
                         "converged": bool(r["converged"])}
            log(f"[bench] davidson solve {name}: {res[name]['time_s']:.1f} s, {r['iterations']} iterations, "
                f"sigma calls {r['n_sigma']}, E={r['energy']:.10f}, residual {r['residual']:.1e}")
        solve = {"tol": 1e-6, "ladder": [list(x) for x in ladder],
                 "note": "residual = ||H u - E u||_2 with FP64 sigma, |u| = 1 (the paper's eigensolver "
                         "tolerance 1e-6); energy = FP64 Rayleigh quotient", **res}
        if "fp64" in res:
            for name in ("mixed", "refined"):
                solve[f"energy_diff_{name}"] = res[name]["energy"] - res["fp64"]["energy"]
                solve[f"speedup_{name}"] = res["fp64"]["time_s"] / res[name]["time_s"]
                log(f"[bench] time to solution: {name} {res[name]['time_s']:.1f} s vs FP64 "
                    f"{res['fp64']['time_s']:.1f} s ({solve[f'speedup_{name}']:.2f}x), "
                    f"|E_{name} - E_FP64| = {abs(solve[f'energy_diff_{name}']):.1e}")
    # Ozaki-scheme sigma: FP64 accuracy from INT8 MFMA digit products
    ozaki = None
    if args.ozaki_steps > 0:
        soz = torch.empty_like(psi)
        t_oz, kto, _ = timed_sigma("ozaki", args.ozaki_steps, 1, soz, True)
        ms_oz = float(np.median(t_oz))
        info_oz = ctx.sigma_info("ozaki")
        kap = int(round((np.sqrt(8 * info_oz["hw_flops"] / info["flops"] + 1) - 1) / 2))
        ms_gemm = (kto["ms_stage1"] + kto["ms_stage2"]) / max(1, kto["calls"])
        int8_tops = info_oz["hw_flops"] * (info["flops"] - kto["flops_pinned"]) / info["flops"] / (ms_gemm * 1e-3) / 1e12
        rel_oz = float((torch.linalg.norm(soz - ref) / torch.linalg.norm(ref)).item())
        e_oz = float(torch.dot(psi, soz).item())
        ozaki = {"slices": kap, "bits": 8 * kap - 1, "ms": ms_oz,
                 "tflops": info["flops"] / (ms_oz * 1e-3) / 1e12,
                 "speedup_vs_fp64": fp64["ms"] / ms_oz if fp64 else None,
                 "sigma_rel_err_vs_fp64": rel_oz, "rayleigh_diff": e_oz - e_ref,
                 "stage1_ms": kto["ms_stage1"] / max(1, kto["calls"]),
                 "stage2_ms": kto["ms_stage2"] / max(1, kto["calls"]),
                 "slicing_ms": kto["ms_convert"] / max(1, kto["calls"]),
                 "pinned_fp64_ms": kto["ms_pinned"] / max(1, kto["calls"]),
                 "int8_tops": int8_tops, "int8_peak_tops": 5000.0, "int8_frac": int8_tops / 5000.0,
                 "roofline": kernel_roofline(kto, "k_gemm_oz", 5000.0, "TOP/s (INT8)",
                                             info_oz["hw_flops"] / info["flops"])}
        log(f"[bench] sigma ozaki ({kap} slices, {8 * kap - 1} bits): median {ms_oz:.1f} ms "
            f"({ozaki['tflops']:.1f} TFLOP/s FP64-equivalent), stage1 {ozaki['stage1_ms']:.1f} + stage2 "
            f"{ozaki['stage2_ms']:.1f} + slicing {ozaki['slicing_ms']:.1f} + pinned {ozaki['pinned_fp64_ms']:.1f} ms; "
            f"INT8 {int8_tops:.0f} TOP/s; |dsigma|/|sigma| = {rel_oz:.2e}")
    su2_leg = None
    if args.su2_steps > 0:
        su2_leg = su2_bench(ctx, args.su2_steps)
    cpu = None
    if not args.no_cpu_baseline:
        t_cpu, t_spent, n_cls, n_terms = cpu_baseline(m, args.cpu_reps)
        cores = len(os.sched_getaffinity(0))
        threads = int(os.environ.get("OMP_NUM_THREADS", cores))
        cpu = {"value": info["flops"] / t_cpu / 1e12, "unit": "TFLOP/s", "cores": min(cores, threads),
               "kind": "oracle",
               "sample": f"the oracle's block-sparse contraction (BlockSparseSigma.apply_matrix, FP64 "
                         f"NumPy) timed on the real enlarged sectors of this {args.config} window for "
                         f"each of its {n_cls} term classes ({args.cpu_reps} repeats, {t_spent:.1f} s "
                         f"timed), with random operators filling every block of the class",
               "model": f"modelled sigma time {t_cpu:.0f} s = sum over classes of the timed time per "
                        f"term x the class's term count ({n_terms} terms); value = the library's "
                        f"algorithmic sigma FLOPs / that time",
               "sigma_s_modelled": t_cpu}
        log(f"[bench] cpu oracle: {t_spent:.1f} s timed over {n_cls} classes -> {t_cpu:.0f} s/sigma modelled")
    peak = PEAK_TFLOPS[args.precision]
    traffic = None
    if args.precision != "fp64" and args.config == "cas54_36":
        csrc = os.path.join(ROOT, "paper_2603_28648_amd", "csrc")
        pt = profiled_traffic("k_gemm_bf16_sigma_cas54_36_D4096.md",
                              [os.path.join(csrc, "kernels_bf16.hip"), os.path.join(csrc, "engine.cpp")],
                              "bf16_launch_config", f"{tuned['stage1']},{tuned['stage2']}")
        if pt is not None:
            traffic = pt[0] / pt[1]  # bytes per chunk-stage launch
    log(f"[bench] HBM traffic per launch from the committed profile: "
        f"{'%.3e bytes' % traffic if traffic else 'none (kernel or configuration differs)'}")
    res = {
        "metric": METRIC,
        "value": tflops,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "bf16": "bf16", "bf16x3": "bf16x3"}[args.precision],
        "data": "synthetic (seeded integral recipe, converged-like random MPS)",
        "config": {"workload": f"{args.config}: K={K} N={N} 2Sz={tsz} D={D} window=({i},{i + 1})",
                   "psi_size": m.psi_size(), "sigma_flops": info["flops"],
                   "sigma_flops_stages": [info["flops_stage1"], info["flops_stage2"]],
                   "sigma_flops_per_term": info["flops_terms"],
                   "stage1_flops_consumed_frac": info["flops_stage1_used"] / max(1.0, info["flops_stage1"]),
                   "pairs": info["n_pairs"], "precision": args.precision,
                   "build_ops_s": round(t_build, 2), "wall_s_timed": round(t_wall, 3),
                   "rayleigh": e_mix, "rayleigh_fp64": e_ref, "rayleigh_diff": e_mix - e_ref,
                   "sigma_rel_err_vs_fp64": rel,
                   "fp64_sigma_ms": fp64["ms"] if fp64 else None,
                   "fp64_sigma_tflops": fp64["tflops"] if fp64 else None,
                   "fp64_frac_of_peak": fp64["frac_of_fp64_peak"] if fp64 else None,
                   "fp64_roofline": fp64["roofline"] if fp64 else None,
                   "speedup_vs_fp64": fp64["ms"] / ms if fp64 else None,
                   "bf16_launch_config": tuned if args.precision != "fp64" else None,
                   "graphs": not args.no_graphs,
                   "bf16_sigma": bf16,
                   "davidson": dav,
                   "davidson_solve": solve,
                   "ozaki": ozaki,
                   "su2": su2_leg},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": f"{kname} (stage-1 and stage-2 grouped-GEMM launches)",
                     "launches_per_step": n_launch / max(1, kt["calls"]),
                     "avg_launch_ms": ms_kernel,
                     "hw_tflops": achieved * (3 if args.precision == "bf16x3" else 1)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
