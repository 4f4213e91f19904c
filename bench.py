"""Benchmark: D3Q19 colour-gradient step at 256^3 in FP32 on one MI355X.

One step = the whole hot path (moments, isotropic gradients, BGK with the
enhanced equilibrium, perturbation, recolouring, streaming) over the whole
lattice.  Input: 32 seeded non-overlapping droplets (radii U[10, 24]) in a
periodic 256^3 box, density ratio 1, tau = 1, A = 0.005, beta = 0.7.

Prints one JSON line with MLUPS, the HBM roofline fraction of the step kernel
(algorithmic 304 B per lattice update / measured kernel time, against 8 TB/s)
and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D3Q19 CG MLUPS + % HBM roofline at 256^3; sweep-serving p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# what the step's machine code and its memory layout are made from: every source of the
# library (not the stream probe) and the build flags
KERNEL_SOURCES = sorted(os.path.relpath(f, os.path.join(ROOT, "paper_2110_05197_amd"))
                        for f in glob.glob(os.path.join(ROOT, "paper_2110_05197_amd", "csrc", "*"))
                        if not f.endswith("stream_probe.hip")) + ["_build.py"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2110_05197_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TRAFFIC_PROFILES = {"D3Q19": "traffic_fused_cg_d3q19_fp32_256.md",
                    "D2Q9": "traffic_fused_cg_d2q9_fp32_4096.md"}


def measured_traffic(lattice: str):
    """HBM bytes per launch of the one-pass CG FP32 step on the lattice's
    benchmark workload, from the committed rocprofv3 counter summary, if it was
    taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_PROFILES[lattice])
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    vals = {}
    for line in txt.splitlines():
        if line.startswith("|") and ":" not in line:
            continue
        for key in ("kernel_sources_sha256_16", "hbm_bytes_per_launch"):
            if line.strip().startswith(key + ":"):
                vals[key] = line.split(":", 1)[1].strip()
    if vals.get("kernel_sources_sha256_16") != kernel_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


MODELS = {"CG": 0, "SC_MP": 1, "SC_MC": 2}
SC_MP_G, SC_MC_GRB = -5.0, 1.2


def shape_of(n: int, lattice: str):
    """D3Q19: n^3.  D2Q9: a square of the same node count (16 n x 16 n at n = 256)."""
    if lattice == "D2Q9":
        L = int(round(n ** 1.5))
        return (1, L, L)
    return (n, n, n)


def workload_fields(n: int, seed: int = 0, model: str = "CG", lattice: str = "D3Q19"):
    from paper_2110_05197_amd import inputs
    shape = shape_of(n, lattice)
    L = shape[2]
    count = 32 if n >= 128 else 4
    rmin, rmax = 10.0 * n / 256, 24.0 * n / 256
    if lattice == "D2Q9":
        count, rmin, rmax = 32, L / 40.0, L / 16.0
    if model == "SC_MP":
        from paper_2110_05197_amd import serve
        liq, gas = serve.sc_coexistence(SC_MP_G)
        rR, rB, _ = inputs.random_droplets(shape, count, rmin, rmax, seed, liq, gas)
        return rR + rB, None
    rR, rB, _ = inputs.random_droplets(shape, count, rmin, rmax, seed)
    if model == "SC_MC":
        return rR + 0.03, rB + 0.03
    return rR, rB


def params(n: int, precision: int = 1, kernel: int = 0, model: str = "CG", lattice: str = "D3Q19",
           conserve: bool = False):
    import paper_2110_05197_amd as M
    nz, ny, nx = shape_of(n, lattice)
    base = dict(lattice=M.D2Q9 if lattice == "D2Q9" else M.D3Q19, precision=precision, nx=nx, ny=ny,
                nz=nz, kernel=kernel)
    if model == "SC_MP":
        return M.make_params(model=M.SC_MP, G=SC_MP_G, tau_R=1.0, rho0_R=2.0, rho0_B=0.15, **base)
    if model == "SC_MC":
        return M.make_params(model=M.SC_MC, G_RB=SC_MC_GRB, tau_R=1.0, tau_B=1.0, rho0_R=1.0,
                             rho0_B=1.0, **base)
    return M.make_params(model=M.CG, rho0_R=1.0, rho0_B=1.0, tau_R=1.0, tau_B=1.0, A=0.005,
                         beta=0.7, conserve_mass=int(conserve), **base)


def stream_probe(n: int):
    """Ceilings of the step's memory pattern: the committed stream probe (built
    next to the library) moving one FP32 D3Q19 step's bytes in each pattern,
    with the population arrays n^3 floats apart and then padded as the
    library pads them."""
    import subprocess
    import paper_2110_05197_amd as M
    exe = os.path.join(ROOT, "paper_2110_05197_amd", "stream_probe")
    if not os.path.exists(exe):
        print("bench.py: stream_probe is not built (run __graft_entry__.build())", file=sys.stderr)
        sys.exit(1)
    words, _, _ = M.population_stride(params(n))
    for pad in (0, words - n ** 3):
        r = subprocess.run([exe, str(n), "20", str(pad)], capture_output=True, text=True, timeout=600)
        sys.stdout.write(r.stdout)
        sys.stdout.flush()
        if r.returncode:
            sys.stderr.write(r.stderr)
            sys.exit(r.returncode)


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo, as lscpu prints it)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(rR, rB, n: int, steps: int, steps_one_thread: int):
    """The FP64 oracle (as it stands: one pass per step over plain arrays,
    OpenMP over the host cores) on `steps` steps of the same fields, built
    here with -O3 -march=native, then on one thread for `steps_one_thread`
    steps.  Each timing includes the oracle's per-call scratch allocation."""
    import tempfile
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle
    tmp = tempfile.mkdtemp(prefix="mclbm_oracle_")
    oracle.use_library(oracle.build_timing(tmp))
    p = oracle.make_params(lattice=1, model=0, nx=n, ny=n, nz=n, rho0_R=1.0, rho0_B=1.0,
                           tau_R=1.0, tau_B=1.0, A=0.005, beta=0.7)
    f0 = oracle.init_equilibrium(p, rR, rB)
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    f = oracle.run(p, f0, steps)
    dt = time.perf_counter() - t0
    del f
    oracle.set_threads(1)
    t0 = time.perf_counter()
    f = oracle.run(p, f0, steps_one_thread)
    dt1 = time.perf_counter() - t0
    del f, f0
    oracle.set_threads(threads)
    return dict(value=n ** 3 * steps / dt / 1e6, unit="MLUPS", cores=threads, kind="oracle",
                sample=f"FP64 oracle, D3Q19 CG {n}^3 of the same 32-droplet fields, {steps} steps on "
                       f"{threads} threads ({dt:.1f} s wall)",
                one_thread=dict(value=n ** 3 * steps_one_thread / dt1 / 1e6, unit="MLUPS",
                                steps=steps_one_thread, wall_s=round(dt1, 1)),
                cpu_model=cpu_model(), build="gcc -O3 -march=native -fopenmp -ffp-contract=off")


def serving_leg(full: bool, conserve: bool = False):
    """Sweep serving: continuous batching (FP32 / mixed, batched graphs) against
    one-at-a-time FP64 solves of the same seeded trace on the same GPU.
    conserve: the batched FP32 / mixed colour-gradient requests keep each
    colour's node mass to one rounding per step."""
    from paper_2110_05197_amd import serve
    if full:
        kw = dict(n=256)
        desc = ("256 requests, Poisson 20/s, CG/SC droplet/ligament, D2Q9 64^2-512^2 / D3Q19 "
                "64^3-160^3, gamma 10^U(0,3), nu ratio 10^U(0,2), sigma 10^U(-3,-1), 1000-20000 steps")
    else:
        kw = dict(n=64, rate=200.0, d2_sizes=(64, 96, 128, 192, 256), d3_sizes=(32, 48, 64, 80, 96),
                  steps_range=(500, 4000))
        desc = ("reduced trace: 64 requests, Poisson 200/s (saturating), CG/SC droplet/ligament, "
                "D2Q9 64^2-256^2 / D3Q19 32^3-96^3, gamma 10^U(0,3), nu ratio 10^U(0,2), "
                "sigma 10^U(-3,-1), 500-4000 steps")
    print(f"[bench] serving: {desc}", file=sys.stderr, flush=True)
    # the full trace runs for minutes: report each finished request
    log = (lambda s: print(s, file=sys.stderr, flush=True)) if full else None
    runs = {}
    for rule in ("fp64", "gamma"):
        trace = serve.make_trace(seed=0, precision_rule=rule, conserve_mass=conserve, **kw)
        done, wall = serve.Server(k_steps=100, log=log, keep_fields=True).run(trace)
        runs[rule] = (done, serve.summarize(done, wall))
        print(f"[bench] batched ({rule} rule): {runs[rule][1]}", file=sys.stderr, flush=True)
    trace2 = serve.make_trace(seed=0, **kw)
    done2, wall2 = serve.serve_one_at_a_time(trace2, log=log, keep_fields=True)
    fifo = serve.summarize(done2, wall2)
    print(f"[bench] one-at-a-time FP64: {fifo}", file=sys.stderr, flush=True)
    by2 = {r.rid: r for r in done2}
    out = dict(trace=desc, trace_is_full=full, conserve_mass=conserve, one_at_a_time_fp64=fifo,
               accuracy_metrics="per request, batched result against its FP64 solve at the final step: "
                                "rho_err = relative max-norm error of rho_R and rho_B; volume_err, jump_err = "
                                "relative difference of the red volume and of the density jump rho_in - rho_out "
                                "across the interface; ekin_ratio_max = largest kinetic-energy ratio")
    for rule, key in (("gamma", "batched_fp32_mixed"), ("fp64", "batched")):
        done, summ = runs[rule]
        serve.compare_runs(done, done2, release_reference=(rule == "fp64"))
        agree = sum(1 for r in done if by2.get(r.rid) is not None and by2[r.rid].outcome == r.outcome)
        acc = serve.accuracy(done)
        print(f"[bench] {key} against the FP64 solves: {acc}", file=sys.stderr, flush=True)
        out[key] = dict(precision=("FP32 below density ratio 100, FP64 from 100" if rule == "fp64"
                                   else "FP32 below density ratio 100, mixed from 100"),
                        **summ, speedup_throughput=round(summ["throughput_req_s"] / fifo["throughput_req_s"], 3),
                        outcome_agreement=f"{agree}/{len(done)}", accuracy_vs_fp64=acc)
    return out


def copy_probe(n: int):
    """A plain copy of the bytes one FP32 step reads (and writes): 38 n^3 floats.
    Counter readings of this kernel scale FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch
    a = torch.ones(38 * n ** 3, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": a.numel() * 4, "launches": 3}))


def _finite(x):
    """The same structure with NaN and infinities as null, so the study and
    sweep lines are strict JSON (an unfitted or diverged case has no value)."""
    if isinstance(x, float):
        return x if math.isfinite(x) else None
    if isinstance(x, dict):
        return {k: _finite(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [_finite(v) for v in x]
    return x


# couplings of the droplet-collision study (Table dropcolParams, set 1), rho_0 = 0.83
MULTIRANGE = dict(G_RB=0.405, Ga_R=-9.0, Ga_B=-8.0, Gr_R=8.1, Gr_B=7.1, psi_rho0=0.83, rho0_X=0.83,
                  rho0_R=1.18, rho0_B=0.18, tau_R=1.0, tau_B=0.8)


def next_rows(n: int, steps: int, reps: int = 20):
    """The multirange Shan-Chen step and the interface observables on the n^3
    workload: time per step or call, HIP events on the library's stream."""
    import torch
    import paper_2110_05197_amd as M
    out = {}
    rR, rB = workload_fields(n, 0)
    frac = rR / (rR + rB)
    N = n ** 3

    def timed(fn, k):
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(k):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    # multirange two-component Shan-Chen (two-pass: the belts reach two nodes)
    p = M.make_params(lattice=M.D3Q19, model=M.SC_MC, precision=M.FP32, nx=n, ny=n, nz=n, **MULTIRANGE)
    sim = M.Sim(p)
    sim.init_equilibrium(0.18 + frac, 0.18 + (1.0 - frac))
    print(f"[bench] multirange step, {n}^3 FP32", file=sys.stderr, flush=True)
    ms = timed(lambda: sim.step(1), steps)
    o = sim.observables()
    bpu = M.bytes_per_update(p)
    # two-pass traffic: the density pass reads the populations and writes drho_R, drho_B, psi_R, psi_B
    # (4 floats), the collide pass reads the populations and that field and writes the populations
    moved = 1.5 * bpu + 2 * 4 * 4
    out["multirange"] = dict(workload=f"SC two-component + multirange forces (Table dropcolParams set 1), {n}^3 periodic, "
                                      "the bench droplets as species A (1.18 / 0.18)",
                             kernel="two-pass (density + collide)", ms_per_step=round(ms, 4),
                             mlups=round(N / (ms * 1e-3) / 1e6, 1), bytes_per_update=bpu,
                             frac_algorithmic=round(bpu * N / (ms * 1e-3) / 8e12, 4),
                             two_pass_bytes_per_update=moved,
                             frac_two_pass_bytes=round(moved * N / (ms * 1e-3) / 8e12, 4),
                             diverged=bool(o["diverged"]))
    sim.close()
    torch.cuda.empty_cache()
    # interface observables on the CG bench state
    p = params(n, 1)
    sim = M.Sim(p)
    sim.init_equilibrium(rR, rB)
    sim.step(100)
    print(f"[bench] interface observables on the {n}^3 CG state", file=sys.stderr, flush=True)
    ms_x = timed(lambda: sim.interface_crossings(0, n // 2, n // 2), reps)
    ms_a = timed(lambda: sim.plane_area(2, n // 2), reps)
    ms_d = timed(lambda: sim.droplets(), 5)
    nd = sim.droplets()
    out["interface"] = dict(workload=f"CG bench state, {n}^3, after 100 steps",
                            crossings_line_ms=round(ms_x, 4), plane_area_ms=round(ms_a, 4),
                            droplets_ms=round(ms_d, 3), droplets_found=int(nd[0]) if isinstance(nd, tuple) else nd,
                            droplets_nodes_per_s=round(N / (ms_d * 1e-3), 1))
    sim.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--precision", type=int, default=1, help="0 FP64, 1 FP32, 2 mixed, 3 FP16")
    ap.add_argument("--kernel", type=int, default=0, help="0 auto (fused), 1 two-pass, 2 fused")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--cpu-steps-one-thread", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the sweep-serving leg")
    ap.add_argument("--serve-full", action="store_true",
                    help="serve the full 256-request trace (minutes) instead of the reduced one")
    ap.add_argument("--conserve-mass", action="store_true",
                    help="CG, FP32 or mixed storage: keep each colour's node mass to one rounding per step "
                         "(the benchmark step and the batched serving requests)")
    ap.add_argument("--next-rows", action="store_true",
                    help="time the multirange Shan-Chen step and the interface observables on the workload")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of one step's population bytes (counter calibration)")
    ap.add_argument("--stream-probe", action="store_true",
                    help="only time the step's memory patterns without stencil or collision (ceilings)")
    ap.add_argument("--sweep", choices=["density", "viscosity", "ekin", "ekin-tau"],
                    help="only run a static-droplet study of the paper (Laplace error, or CG vs SC "
                         "spurious-current energy over sigma) as one GPU batch")
    ap.add_argument("--sweep-steps", type=int, default=100_000)
    ap.add_argument("--sweep-serve", action="store_true",
                    help="run the Laplace sweep's droplets as requests of the sweep server")
    ap.add_argument("--model", default="CG", choices=sorted(MODELS))
    ap.add_argument("--lattice", default="D3Q19", choices=["D3Q19", "D2Q9"])
    ap.add_argument("--study", choices=["rp", "ligament", "oscillation", "contraction", "dropOsc", "drift"],
                    help="physics run of a paper case instead of the benchmark: the Rayleigh-Plateau jet "
                         "(CG and SC, breakup and satellites), the density-ratio-1000 ligament "
                         "(mixed and FP16 storage), the 128^3 oscillating droplet (FP32 and FP64) or the "
                         "ligament contraction sets of Table contrParams (CG and SC), or the droplet "
                         "oscillations of Table dropOscParams at R_D = 12-49 (CG and SC)")
    ap.add_argument("--study-steps", type=int, default=None)
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.size)
        return
    if args.next_rows:
        print(json.dumps(next_rows(args.size, args.steps)))
        return
    if args.stream_probe:
        stream_probe(args.size)
        return
    if args.study:
        import paper_2110_05197_amd as M
        from paper_2110_05197_amd import studies
        log = lambda *a: print(*a, file=sys.stderr, flush=True)
        if args.study == "drift":
            n = args.size
            rR, rB = workload_fields(n, 0, args.model, args.lattice)
            out = dict(study="mass-drift", workload=f"{args.lattice} {args.model} {n}^3 periodic, 32 seeded droplets",
                       precision=args.precision,
                       run=studies.mass_drift(M, params(n, args.precision, args.kernel, args.model, args.lattice),
                                              rR, rB, steps=args.study_steps or 10000, log=log))
        elif args.study == "rp":
            steps = args.study_steps or 30000
            sc = studies.sc_mc_sigma(M)
            log(f"[rp] Shan-Chen sigma {sc['sigma']:.4f} (Laplace, R = {sc['radius']:.2f})")
            out = dict(study="rayleigh-plateau", sc_mc_sigma=sc,
                       runs=[studies.rayleigh_plateau(M, m, steps=steps, sigma=sc["sigma"], log=log)
                             for m in ("CG", "SC_MC")])
        elif args.study == "dropOsc":
            out = dict(study="droplet-oscillation", runs=studies.oscillation_table(M, log=log))
        elif args.study == "contraction":
            out = dict(study="ligament-contraction", runs=studies.ligament_contraction(M, log=log))
        elif args.study == "oscillation":
            steps = args.study_steps or 20000
            out = dict(study="oscillation", runs=[studies.oscillation(M, prec, steps=steps, log=log)
                                                  for prec in (M.FP32, M.FP64)])
        else:
            steps = args.study_steps or 40000
            out = dict(study="ligament", runs=[studies.ligament(M, prec, steps=steps, log=log)
                                               for prec in (M.MIXED, M.FP16)])
        print(json.dumps(_finite(out)))
        return
    if args.sweep:
        from paper_2110_05197_amd import sweeps
        out = sweeps.run(args.sweep, steps=args.sweep_steps, via_server=args.sweep_serve,
                         log=lambda *a: print(*a, file=sys.stderr, flush=True))
        print(json.dumps(_finite(out)))
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); the "
              "multi-GPU slab decomposition is a design, not an implementation.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2110_05197_amd as M
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    n = args.size
    headline = args.model == "CG" and args.lattice == "D3Q19"
    print(f"[bench] generating {args.lattice} {args.model} fields ({n}^3 = "
          f"{'x'.join(str(d) for d in shape_of(n, args.lattice)[::-1] if d > 1)} nodes)",
          file=sys.stderr, flush=True)
    rR, rB = workload_fields(n, 0, args.model, args.lattice)
    p = params(n, args.precision, args.kernel, args.model, args.lattice, args.conserve_mass)
    sim = M.Sim(p)
    sim.init_equilibrium(rR, rB)
    stream = torch.cuda.current_stream()
    o0 = sim.observables()
    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    st, done = sim.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    ms = ms_total / args.steps
    o1 = sim.observables()
    N = p["nx"] * p["ny"] * p["nz"]
    mlups = N / (ms * 1e-3) / 1e6
    bpu = M.bytes_per_update(p)
    achieved = bpu * N / (ms * 1e-3) / 1e9
    fused = sim.kernel_used() == M.KERNEL_FUSED
    drift = abs(o1["mass_R"] - o0["mass_R"]) / o0["mass_R"] if o0["mass_R"] else 0.0
    print(f"[bench] {ms:.4f} ms/step, {mlups:.0f} MLUPS, {achieved:.0f} GB/s algorithmic, "
          f"mass drift {drift:.2e}, diverged={o1['diverged']}", file=sys.stderr, flush=True)
    traffic = (measured_traffic(args.lattice)
               if (fused and args.model == "CG" and args.precision == 1 and n == 256) else None)
    del sim
    torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline and headline:
        print(f"[bench] cpu baseline ({args.cpu_steps} oracle steps)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(rR, rB, n, args.cpu_steps, args.cpu_steps_one_thread)

    serving = None
    if not args.no_serve:
        serving = serving_leg(args.serve_full, args.conserve_mass)

    dtype = {0: "f64", 1: "f32", 2: "f32+f64", 3: "f16-storage/f32"}[args.precision]
    out = {
        "metric": METRIC if headline else f"{args.lattice} {args.model} MLUPS + % HBM roofline",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": (f"D3Q19 colour-gradient step, {n}^3 periodic, 32 seeded droplets r~U[10,24], "
                         "gamma=1, tau=1, A=0.005, beta=0.7") if headline else
                        (f"{args.lattice} {args.model} step, {p['nx']}x{p['ny']}x{p['nz']} periodic, 32 seeded "
                         "droplets" + (f", G={SC_MP_G} at coexistence" if args.model == "SC_MP" else "")
                         + (f", G_RB={SC_MC_GRB}" if args.model == "SC_MC" else "")),
            "lattice": args.lattice, "model": args.model, "nx": p["nx"], "ny": p["ny"], "nz": p["nz"],
            "precision": dtype, "kernel": "fused one-pass" if fused else "two-pass",
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_update": bpu,
        },
        "cpu_baseline": cpu,
        "mass_drift": drift,
        "serving": serving,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
