"""Benchmark: BRDF solves per second (Fourier orders x incident directions) on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload batched] [--no-cpu-baseline]

A step is one full solve of the workload (all stages: Legendre matrices and E/F assembly, FE
product, eigen-decomposition and its refinement, mode vectors, boundary solves, emergent response
and Fourier synthesis of F_r) with the inputs already resident in device memory. The unit count of
a layer is M x N x n_dphi (orders x incident zenith nodes x incident azimuths). The default
workload is the largest one: 256 layers of uneven N in {16, 24, 32, 48, 64} with L = M = n_dphi = 2N.
Prints one JSON line.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector and FP64 matrix
PEAK_HBM_GBS = 8000.0
GOLDEN = os.path.join(ROOT, "tests", "golden")


def stage_work(stage, layers):
    """Algorithmic work of one launch of `stage` over all (layer, order) items.

    Returns (bound, amount, unit) with amount in flops (alu/mfma) or bytes (hbm)."""
    fl = 0.0
    by = 0.0
    for N, L, M, P in zip(layers.N, layers.L, layers.M, layers.n_dphi):
        n = 4 * N
        for m in range(M):
            if stage == "eigen":
                fl += 25.0 * n ** 3           # real Schur form + eigenvectors (Golub-Van Loan count)
            elif stage in ("gemm_FE", "gemm_U", "gemm_V"):
                fl += 2.0 * n ** 3
            elif stage == "refine":
                fl += 6.0 * n ** 3 + 2.0 / 3.0 * n ** 3 + 2.0 * n ** 3  # three GEMMs, LU of U^T, right division
            elif stage == "hqapply":
                fl += 2.0 * n ** 3                           # n - 2 reflectors applied to n columns
            elif stage == "lu":
                fl += 2 * (2.0 / 3.0 * n ** 3)               # LU of S' and T'
            elif stage == "trsm":
                fl += 2 * (2.0 * n ** 3)                     # two n-RHS right divisions
            elif stage == "assemble":
                fl += N * N * (L - m) * 72.0  # 36 products-with-coefficient per degree and block pair
        if stage == "synth":
            by += 8.0 * (M * n * n + N * N * P * 16)
    if stage == "synth":
        return "hbm", by, "GB/s"
    if stage in ("gemm_FE", "gemm_U", "gemm_V"):
        return "mfma", fl, "TFLOP/s"
    return "alu", fl, "TFLOP/s"


KERNEL_SOURCE = {"k_eigen": "k_eigen.hip", "k_eigen_big": "k_eigen.hip", "k_hqapply": "k_eigen.hip", "k_hqapply_mfma": "k_eigen.hip", "k_lu": "k_bc.hip", "k_trsm": "k_bc.hip", "k_vfix": "k_bc.hip",
                 "k_bcbuild": "k_bc.hip", "k_colscal": "k_bc.hip", "k_response": "k_bc.hip", "k_gemm": "k_gemm.hip",
                 "k_assemble": "k_assemble.hip", "k_legendre": "k_assemble.hip", "k_validate": "k_assemble.hip",
                 "k_synth": "k_synth.hip", "k_synth_mfma": "k_synth.hip", "k_refine": "k_refine.hip"}


def stage_kernels(stage):
    """Kernels whose launches make up a stage (the eigen stage launches one kernel for the systems
    held in LDS and one for the larger ones)."""
    if stage.startswith("gemm"):
        return ["k_gemm"]
    if stage == "eigen":
        return ["k_eigen", "k_eigen_big"]
    return [f"k_{stage}"]


def measured_traffic(kernels, workload):
    """HBM bytes per launch of the stage made of `kernels`, summed over the kernels recorded in the
    byte counters of this workload (profiles/traffic_<workload>.txt); None when there is no record
    or a recorded kernel's sources have changed since it was taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path) or any(k not in KERNEL_SOURCE for k in kernels):
        return None
    rec = {}
    with open(path) as fh:
        for line in fh:
            f = line.split()
            if len(f) == 5 and f[0] in kernels:
                rec[f[0]] = (f[1], float(f[4]))
    if not rec:
        return None
    total = 0.0
    for k, (sha_rec, nbytes) in rec.items():
        h = hashlib.sha256()
        for part in (KERNEL_SOURCE[k], "vbrdf_internal.hpp"):
            with open(os.path.join(ROOT, "paper_1707_05882_amd", "csrc", part), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest()[:16] != sha_rec:
            return None
        total += nbytes
    return total


def golden_samples(name):
    """Stored oracle values for the workload: list of (layer, azimuth indices, F sample, scale).

    The files are written by the scripts next to them, which call only the CPU oracle."""
    base = name.split("_")[0]
    path = os.path.join(GOLDEN, f"{base}_sample.npz")
    if not os.path.exists(path):
        return []
    g = np.load(path)
    if "layers" in g:
        return [(int(i), g[f"az{i}"], g[f"F{i}"], float(g[f"scale{i}"])) for i in g["layers"]]
    return [(0, g["az"], g["F"], float(g["scale"]))]


def err_vs_oracle(F, layers, name):
    """max |F - F_oracle| / max |F_oracle,II| over the stored samples (every node pair at a few
    azimuths), per layer, maximum over the sampled layers; None without stored samples."""
    samples = golden_samples(name)
    if not samples:
        return None, 0
    offs = np.cumsum([0] + [n * n * p * 16 for n, p in zip(layers.N, layers.n_dphi)])
    worst = 0.0
    for i, az, Fo, scale in samples:
        n, p = layers.N[i], layers.n_dphi[i]
        Fl = F[offs[i]:offs[i + 1]].view(n, n, p, 4, 4)[:, :, list(int(a) for a in az)].cpu().numpy()
        worst = max(worst, float(np.abs(Fl - Fo).max() / scale))
    return worst, len(samples)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(layers, units):
    """The CPU oracle on a bounded, stated sample of the workload, scaled to the whole job.

    One layer per distinct N (the first of each), every s-th Fourier order of it (s chosen so that
    the sample is about 10 s of work); the per-layer time is the sampled orders' solve and synthesis
    time times M / (orders sampled), and the job time weights each N by its number of layers. The
    same sample at one BLAS thread, with a wider order stride, gives the single-thread rate."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import dom
    from oracle.quadrature import double_gauss

    firsts = {}
    for i, N in enumerate(layers.N):
        firsts.setdefault(N, i)
    count = {N: layers.N.count(N) for N in firsts}
    nmax = max(firsts)
    work_per_order = {N: (4 * N) ** 3 for N in firsts}

    def run(stride_at_max):
        total = 0.0
        detail = []
        for N, i in sorted(firsts.items()):
            M = layers.M[i]
            # smaller systems are cheaper per order: sample them more densely
            s = max(1, int(round(stride_at_max * work_per_order[N] / work_per_order[nmax])))
            s = min(s, M)
            ms = list(range(0, M, s))
            coef, om = dom.validate(layers.coef[i], layers.tau[i], layers.omega[i], N, M)
            mu, al = double_gauss(N)
            t0 = time.perf_counter()
            R = [dom.solve_order(coef, om, layers.tau[i], m, mu, al) for m in ms]
            dom.synthesize(R, mu, layers.n_dphi[i])
            dt = time.perf_counter() - t0
            total += dt * M / len(ms) * count[N]
            detail.append(f"N={N}: {len(ms)}/{M} orders")
        return total, detail

    # stride at the largest N so that the all-threads sample is roughly 10 s
    big = firsts[nmax]
    probe_m = 0
    coef, om = dom.validate(layers.coef[big], layers.tau[big], layers.omega[big], nmax, layers.M[big])
    mu, al = double_gauss(nmax)
    t0 = time.perf_counter()
    dom.solve_order(coef, om, layers.tau[big], probe_m, mu, al)
    t_order = time.perf_counter() - t0
    per_sweep = t_order * sum(layers.M[i] * work_per_order[N] / work_per_order[nmax] for N, i in firsts.items())
    stride = max(1, int(np.ceil(per_sweep / 8.0)))
    t_all, detail = run(stride)
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    with threadpool_limits(limits=1):
        t_one, detail1 = run(stride * 4)
    return {"value": units / t_all, "unit": "BRDF solves/s", "cores": int(threads), "kind": "oracle",
            "sample": (f"one layer per N ({', '.join(detail)}), scaled by M / sampled orders and by the "
                       f"number of layers of each N; whole-job estimate {t_all:.1f} s"),
            "one_thread": {"value": units / t_one, "cores": 1, "sample": ", ".join(detail1)},
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched")
    ap.add_argument("--graph-steps", type=int, default=5, help="replays of the hipGraph timed beside the headline")
    ap.add_argument("--precision", choices=["fp64", "fp32_refined"], default="fp64",
                    help="arithmetic of the boundary solves of the timed path")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default schedule and tile shape instead of running the autotuner first")
    ap.add_argument("--compare-steps", type=int, default=3,
                    help="solves of the other precision timed for the comparison block (0: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch

        x = torch.ones(args.copy_probe * 2 ** 17, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": x.numel() * 8, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (orders and layers are "
              "independent, so a multi-GPU run would shard them; that path is not built).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1707_05882_amd import binding
    from paper_1707_05882_amd.api import pack_coefficients
    from workloads import workload

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    layers = workload(args.workload)
    units = layers.units()
    prec_code = {"fp64": binding.PRECISION_FP64, "fp32_refined": binding.PRECISION_FP32_REFINED}
    t_plan = time.perf_counter()
    plan = binding.Plan(layers.N, layers.L, layers.M, layers.n_dphi, precision=prec_code[args.precision],
                        flags=binding.FLAG_STAGE_TIMING)
    plan_ms = (time.perf_counter() - t_plan) * 1e3
    tau = torch.as_tensor(layers.tau, device=dev)
    omega = torch.as_tensor(layers.omega, device=dev)
    coef = torch.as_tensor(pack_coefficients(layers.coef), device=dev)
    F = torch.empty(plan.output_bytes() // 8, dtype=torch.float64, device=dev)
    status = torch.empty(layers.n_layers, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)

    tuning = None
    if not args.no_autotune:  # the library's autotuner picks the eigensolver schedule and tile shape
        tuning = plan.autotune(tau, omega, coef, F, status, stream.cuda_stream)
        print(f"autotuned: {tuning}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        plan.solve(tau, omega, coef, F, status, stream.cuda_stream)
    torch.cuda.synchronize()
    if args.warmup:
        plan.stage_times()  # discard warm-up events
    st = status.cpu().numpy()
    if np.any(st != 0):
        print(f"solve failed: layer status {st.tolist()}", file=sys.stderr)
        sys.exit(1)
    print(f"warm-up done ({args.warmup} solves), timing {args.steps}", file=sys.stderr, flush=True)

    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(args.steps):
        plan.solve(tau, omega, coef, F, status, stream.cuda_stream)
    t1.record(stream)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    stages = plan.stage_times()
    ms = total_ms / args.steps
    if np.any(status.cpu().numpy() != 0) or not torch.isfinite(F).all():
        print("solve failed during the timed region", file=sys.stderr)
        sys.exit(1)
    err, n_checked = err_vs_oracle(F, layers, layers.name)

    # the same solve captured once into a hipGraph and replayed (launch overhead removed); reported
    # beside the headline, which is the stage-timed eager sequence above
    graph_ms = None
    gsteps = max(1, min(args.graph_steps, args.steps))
    try:
        gplan = binding.Plan(layers.N, layers.L, layers.M, layers.n_dphi, precision=prec_code[args.precision],
                             flags=binding.FLAG_GRAPH)
        if tuning:
            gplan.set_tuning(tuning["eigen_schedule"], tuning["trsm_rows"])
        gstream = torch.cuda.Stream()
        Fg = torch.empty_like(F)
        with torch.cuda.stream(gstream):
            gplan.solve(tau, omega, coef, Fg, status, gstream.cuda_stream)
            gstream.synchronize()
            g0 = torch.cuda.Event(enable_timing=True)
            g1 = torch.cuda.Event(enable_timing=True)
            g0.record(gstream)
            for _ in range(gsteps):
                gplan.solve(tau, omega, coef, Fg, status, gstream.cuda_stream)
            g1.record(gstream)
        torch.cuda.synchronize()
        if torch.equal(Fg, F):
            graph_ms = g0.elapsed_time(g1) / gsteps
        gplan.close()
    except binding.VbrdfError as e:
        print(f"graph replay unavailable: {e}", file=sys.stderr)

    # the other precision on the same inputs: a few timed solves and its error against the oracle
    compare = None
    if args.compare_steps > 0:
        other = "fp32_refined" if args.precision == "fp64" else "fp64"
        cplan = binding.Plan(layers.N, layers.L, layers.M, layers.n_dphi, precision=prec_code[other])
        if tuning:
            cplan.set_tuning(tuning["eigen_schedule"], tuning["trsm_rows"])
        Fc = torch.empty_like(F)
        sc = torch.empty_like(status)
        cplan.solve(tau, omega, coef, Fc, sc, stream.cuda_stream)
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        for _ in range(args.compare_steps):
            cplan.solve(tau, omega, coef, Fc, sc, stream.cuda_stream)
        c1.record(stream)
        torch.cuda.synchronize()
        cms = c0.elapsed_time(c1) / args.compare_steps
        cerr, _ = err_vs_oracle(Fc, layers, layers.name)
        compare = {"precision": other, "ms_per_step": cms, "value": units / (cms / 1e3),
                   "err_vs_oracle": cerr, "status_ok": bool((sc.cpu().numpy() == 0).all()),
                   "speedup_of_headline": cms / ms}
        cplan.close()
        del Fc

    dom_stage = max(stages, key=stages.get)
    bound, work, unit = stage_work(dom_stage, layers)
    dur_s = stages[dom_stage] / 1e3
    if bound == "hbm":
        achieved, peak = work / dur_s / 1e9, PEAK_HBM_GBS
    else:
        achieved, peak = work / dur_s / 1e12, PEAK_FP64_TFLOPS
    kernels = stage_kernels(dom_stage)
    roofline = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
                "traffic": measured_traffic(kernels, layers.name), "kernel": "+".join(kernels),
                "stage_ms": {k: round(v, 4) for k, v in stages.items()}}
    one = layers.n_layers == 1
    out = {
        "metric": "BRDF solves/sec (orders x incident dirs)",
        "value": units / (ms / 1e3),
        "unit": "BRDF solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": layers.name, "layers": layers.n_layers,
                   "N": layers.N[0] if one else sorted(set(layers.N)),
                   "L": layers.L[0] if one else "2N", "M": layers.M[0] if one else "2N",
                   "n_dphi": layers.n_dphi[0] if one else "2N", "units_per_step": units,
                   "precision": args.precision, "base": "black"},
        "err_vs_oracle": err,
        "err_layers_checked": n_checked,
        "physical_rhs_per_s": sum(m * 4 * n for m, n in zip(layers.M, layers.N)) / (ms / 1e3),
        "plan_ms": plan_ms,
        "tuning": tuning,
        "roofline": roofline,
        "graph_ms_per_step": graph_ms,
        "compare": compare,
    }
    if not args.no_cpu_baseline:
        print("timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(layers, units)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
