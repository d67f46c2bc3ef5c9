"""Benchmark of the time-spectral GLS hot path on one MI355X.

Workload (default): synthetic Fontan-like cross junction, ~1M P1 tets,
K = 6 harmonics (the paper's 7 modes), Re = 500, Wo = 10, seeded k^-2 inflow
waveforms, zero-traction outlets with backflow stabilization, FP64.

One step = one Newton iteration of the whole hot path through the C ABI:
linearize (nodal time samples, tau eigen-solves at every quadrature point,
residual), Jacobi diagonal, one GMRES cycle of a fixed number of tangent
products with Gram-Schmidt, update.  `value` counts the tangent products'
degree-of-freedom-modes processed per second of the whole step:
steps * jv_per_step * n_nodes * 4 * (2K+1) / seconds / 1e9.

Also reported: the element kernel's roofline position (FP64 ALU bound) from
per-launch HIP events recorded inside the library over the timed region, the
pure tangent-product rate, and the oracle timed on a bounded sample of the
same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Jv GDOF-modes/s; time-to-1e-8 residual, plain FP64 vs mixed/learned/batched"
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def jv_flops_per_element(K: int, variant: str = "picard") -> float:
    """Algorithmic FP64 flops of one tangent product per element: the DFT
    rows of the sampled products (2nM each; 81 rows per element for the
    Picard tangent, 114 for the Newton one), the packed tau apply (24 n^2)
    and the modal element algebra (~300 n)."""
    n, M = 2 * K + 1, 3 * K + 1
    R = 81 if variant != "newton" else 114
    return 2.0 * n * M * R + 24.0 * n * n + 300.0 * n


def jv_bytes(K: int, E: int, nn: int, variant: str = "picard", word: int = 8) -> float:
    """Algorithmic HBM bytes of one tangent product: packed tau (4 points x
    n(n+1)/2), element connectivity + geometry (4 i32 + 13 f64), and per node
    the direction in, the frozen state and the product out; word = 8 for the
    FP64 tangent, 4 for the FP32 one (tau, state and direction in FP32)."""
    n = 2 * K + 1
    P = n * (n + 1) // 2
    b = E * (4.0 * word * P + 120.0) + nn * word * (4 * n + 3 * n + 4 * n)
    if variant == "newton":
        b += E * 12.0 * word * n
    return b


def _workload(name):
    from workloads import junction_problem, womersley_problem
    if name == "junction_1M_K6":
        return junction_problem(h=0.048, K=6, Re=500.0, Wo=10.0, seed=0), dict(
            workload="junction_1M_K6", geometry="cross junction: inlets r=0.8 (-z), 0.6 (+z); "
            "outlets r=0.5 (+-x); arms 4", h=0.048, K=6, Re=500.0, Wo=10.0, seed=0)
    if name == "womersley_6k_K3":
        return womersley_problem(4, 16, K=3), dict(
            workload="womersley_6k_K3", geometry="pipe R=1 L=4", K=3, Re=100.0, Wo=5.0)
    raise SystemExit(f"unknown workload {name}")


def _oracle_patch(prob, first, n_sample):
    """Elements [first, first + n_sample) (Morton order: a contiguous patch)
    as a stand-alone oracle problem with its seeded state and direction."""
    import numpy as np
    import oracle as O
    tets = prob.mesh.tets[first:first + n_sample]
    used = np.unique(tets)
    remap = -np.ones(prob.mesh.n_nodes, dtype=np.int64)
    remap[used] = np.arange(used.size)
    dn = remap[prob.dirichlet_nodes]
    par = O.Params(K=prob.K, rho=prob.rho, mu=prob.mu, omega=prob.omega, C_I=prob.C_I,
                   backflow_beta=prob.backflow_beta, dirichlet_nodes=dn[dn >= 0],
                   neumann_tris=np.zeros((0, 3), np.int32))
    rng = np.random.default_rng(first)
    y = rng.standard_normal((used.size, 4, 2 * prob.K + 2)) * 0.1
    v = rng.standard_normal(y.shape)
    return par, prob.mesh.xyz[used], remap[tets].astype(np.int32), y, v


def _oracle_step_seconds(task):
    """Wall time of one oracle Newton step's work (linearize, Jacobi diagonal,
    jv_per_step Picard products) on one patch, BLAS limited to one thread;
    a first untimed run absorbs start-up (process pool worker)."""
    par, xyz, t, y, v, jv_per_step, runs = task
    from threadpoolctl import threadpool_limits
    import oracle as O

    def one():
        w0 = time.perf_counter()
        lin = O.linearize(par, xyz, t, y)
        O.jacobian_diagonal(par, xyz, t, lin)
        for _ in range(jv_per_step):
            O.jv(par, xyz, t, lin, v, "picard")
        return time.perf_counter() - w0

    with threadpool_limits(limits=1):
        return [one() for _ in range(runs)]


def cpu_baseline(prob, jv_per_step, n_sample=1200, repeats=3):
    """The oracle (as it stands: NumPy, effectively one thread per process)
    on bounded samples of the same workload, scaled to the full mesh.

    * 1 core: one process, `repeats` runs on one patch of n_sample elements
      (median).
    * all cores: one worker process per core the process may use (CPU
      affinity mask, at most 16), each on its own patch, `repeats` timed runs
      after an untimed one; the rate is total elements / the slowest
      worker's median run."""
    import multiprocessing as mp
    cores = min(len(os.sched_getaffinity(0)), 16)
    patches = [_oracle_patch(prob, i * n_sample, n_sample) for i in range(cores)]
    one = sorted(_oracle_step_seconds(patches[0] + (jv_per_step, repeats + 1))[1:])
    med_one = one[repeats // 2]
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_step_seconds, [pt + (jv_per_step, repeats + 1) for pt in patches])
    med_workers = [sorted(r[1:])[repeats // 2] for r in res]
    wall_all = max(med_workers)
    scale = prob.mesh.n_tets / n_sample
    dof = prob.mesh.n_nodes * 4 * (2 * prob.K + 1)
    rate_one = jv_per_step * dof / (med_one * scale) / 1e9
    rate_all = rate_one * med_one / wall_all * cores
    return dict(value=rate_all, unit="GDOF-modes/s", cores=cores, kind="oracle",
                value_1core=rate_one,
                sample=f"oracle Newton-step work (linearize, Jacobi diagonal, {jv_per_step} Picard "
                       f"tangent products) on patches of {n_sample} of {prob.mesh.n_tets} elements, "
                       f"scaled by {scale:.0f}x to the full mesh; 1 core: median of {repeats} runs "
                       f"({med_one:.2f} s); {cores} cores: {cores} worker processes on their own "
                       f"patches, slowest median {wall_all:.2f} s",
                seconds_1core=[round(w, 3) for w in one],
                seconds_per_worker=[round(w, 3) for w in med_workers])


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_op_junction_1M_K6_traffic.txt")
KERNEL_SOURCES = ["paper_2311_09465_amd/csrc/elemop.hip", "paper_2311_09465_amd/csrc/elem.hip",
                  "paper_2311_09465_amd/csrc/common.cuh", "paper_2311_09465_amd/csrc/internal.h"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_tau_counted():
    """tau's counted FP64 flops per launch, rate and fraction of the FP64 peak
    (VALU + MFMA counters over the same dispatches' cycles) from the committed
    instruction-issue summary, or None when it is missing or was taken for
    other kernel sources."""
    try:
        txt = open(ISSUE_FILE).read()
        if f"kernel_source_hash = {kernel_source_hash()}" not in txt:
            return None
        sec = txt.split("[k_tau]", 1)[1].split("\n[", 1)[0]
        kv = {}
        for line in sec.splitlines():
            if "=" in line:
                k, v = line.split("=", 1)
                kv[k.strip()] = v.split("(")[0].strip()
        return dict(flops_per_launch=float(kv["fp64_flops_counted_per_dispatch"]),
                    tflops=float(kv["fp64_tflops_counted"]),
                    frac=float(kv["frac_fp64_peak_counted"]),
                    launch_us=float(kv["kernel_cycles"]) / 2.4e3)
    except (OSError, IndexError, ValueError, KeyError):
        return None


def read_traffic():
    """HBM bytes per launch of the tangent element kernel from the committed
    rocprofv3 counter summary, or None when that summary is missing or was
    taken for a different version of the kernel sources."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if "=" in line and not line.startswith(("#", " ")):
                    k, v = line.split("=", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_source_hash") != kernel_source_hash():
            return None
        return dict(bytes_per_launch=float(kv["hbm_bytes_per_launch"]),
                    fetch_bytes=float(kv["fetch_bytes_per_launch"]),
                    write_bytes=float(kv["write_bytes_per_launch"]),
                    f32_bytes_per_launch=float(kv["f32_hbm_bytes_per_launch"]))
    except (OSError, KeyError, ValueError):
        return None


def probe(args):
    """Counter-collection workload at the benchmark's state: the warm-up
    Newton steps of the benchmark (each linearizes: tau at the states the
    timed steps see), three FP64 and three FP32 tangent products, then a
    plain device copy of 512 MiB (the reference for scaling the counters)."""
    import torch
    import paper_2311_09465_amd as T
    from workloads import initial_guess
    prob, _ = _workload(args.workload)
    s = T.Solver.from_problem(prob)
    y = torch.from_numpy(initial_guess(prob)).cuda()
    m = args.jv_per_step
    if args.warmup > 0:
        s.solve(y, max_newton=args.warmup, rtol=1e-300, lin_rtol=1e-300, restart=m, max_matvec=m,
                jacobian=args.jacobian)
    s.linearize(y)
    v = torch.randn_like(y)
    o = torch.zeros_like(y)
    for _ in range(3):
        s.jv(v, o, args.jacobian)
    for _ in range(3):
        s.jv(v, o, args.jacobian, precision="f32")
    a = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print("probe done", flush=True)


def summarize_pmc(fetch_csv, write_csv, command):
    """Writes the traffic summary from two rocprofv3 --pmc CSV files
    (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), scaled by what the same
    counters read for the 512 MiB copy of the probe."""
    import csv

    def per_kernel(path, counter):
        rows = list(csv.DictReader(open(path)))
        out = []
        for r in rows:
            if r["Counter_Name"] == counter:
                out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"]) * 1024.0))
        return out

    copy_bytes = float(64 << 20) * 8.0
    res = {}
    for path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        rows = per_kernel(path, counter)
        cp = [r for r in rows if "copy" in r[1].lower()]
        if not cp:
            raise SystemExit(f"{path}: copy dispatch not found")
        copy_meas = max(r[2] for r in cp)
        factor = copy_bytes / copy_meas
        for typ in ("double", "float"):
            op = [r for r in rows if "k_op<" in r[1] and f", 0, {typ}>" in r[1]]
            if not op:
                raise SystemExit(f"{path}: k_op<K, 0, {typ}> dispatch not found")
            raw = op[-1][2]
            res[(counter, typ)] = (raw, factor, raw * factor, copy_meas)
    fb, wb = res[("FETCH_SIZE", "double")][2], res[("WRITE_SIZE", "double")][2]
    fb32, wb32 = res[("FETCH_SIZE", "float")][2], res[("WRITE_SIZE", "float")][2]
    lines = [
        "# HBM traffic of the tangent element kernel k_op<6,0,T> (junction 1M tets, K = 6),",
        "# T = double (FP64 tangent) and T = float (mixed-precision tangent, f32_ lines)",
        "# Commands (repository root, one MI355X):",
        f"#   {command.format(counter='FETCH_SIZE', d='pmc_fetch')}",
        f"#   {command.format(counter='WRITE_SIZE', d='pmc_write')}",
        f"#   python bench.py --summarize-pmc <pmc_fetch csv> <pmc_write csv>",
        "# Counters are KiB per dispatch; each is scaled by (bytes of the 512 MiB probe copy) /",
        "# (what the same counter reads for that copy).",
        f"fetch_raw_bytes = {res[('FETCH_SIZE', 'double')][0]:.0f}",
        f"fetch_copy_factor = {res[('FETCH_SIZE', 'double')][1]:.4f}",
        f"write_raw_bytes = {res[('WRITE_SIZE', 'double')][0]:.0f}",
        f"write_copy_factor = {res[('WRITE_SIZE', 'double')][1]:.4f}",
        f"fetch_bytes_per_launch = {fb:.0f}",
        f"write_bytes_per_launch = {wb:.0f}",
        f"hbm_bytes_per_launch = {fb + wb:.0f}",
        f"f32_fetch_raw_bytes = {res[('FETCH_SIZE', 'float')][0]:.0f}",
        f"f32_write_raw_bytes = {res[('WRITE_SIZE', 'float')][0]:.0f}",
        f"f32_fetch_bytes_per_launch = {fb32:.0f}",
        f"f32_write_bytes_per_launch = {wb32:.0f}",
        f"f32_hbm_bytes_per_launch = {fb32 + wb32:.0f}",
        f"kernel_source_hash = {kernel_source_hash()}",
    ]
    with open(TRAFFIC_FILE, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


ISSUE_FILE = os.path.join(ROOT, "profiles", "k_op_junction_1M_K6_issue.txt")
ISSUE_PASSES = (
    "SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_INST_ANY SQ_WAIT_INST_LDS SQ_ACTIVE_INST_VALU "
    "SQ_ACTIVE_INST_LDS SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE",
    "SQ_INSTS_VALU SQ_INSTS_MFMA SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_INSTS_VALU_MFMA_MOPS_F64 "
    "SQ_INSTS_VALU_FLOPS_FP64 SQ_ACTIVE_INST_VMEM SQ_WAIT_ANY",
    "SQ_INSTS_SALU SQ_INSTS_SMEM SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_INSTS_VALU_MFMA_MOPS_F32 "
    "SQ_INSTS_VALU_FLOPS_FP32 SQ_ACTIVE_INST_SCA SQ_INSTS_BRANCH",
)


def summarize_issue(csvs):
    """Instruction-issue summary of the tangent element kernel (and tau and
    the gather) from three rocprofv3 --pmc CSV files of the probe workload:
    per-dispatch averages, per element, and per SIMD as fractions of the
    kernel's cycles (GRBM_GUI_ACTIVE is summed over the 8 XCDs; 1,024 SIMDs;
    SQ_WAVE_CYCLES, SQ_WAIT_* and SQ_ACTIVE_INST_* count 4-cycle units;
    an FP64 16x16x4 MFMA occupies its SIMD's matrix unit for 64 cycles)."""
    import csv
    import collections
    prob, _ = _workload("junction_1M_K6")
    E = prob.mesh.n_tets
    tot = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    for path in csvs:
        for r in csv.DictReader(open(path)):
            k = r["Kernel_Name"]
            tot[k][r["Counter_Name"]] += float(r["Counter_Value"])
            disp[(k, path)].add(int(r["Dispatch_Id"]))
    want = [("k_op<6, 0, double>", "k_op FP64 tangent"), ("k_op<6, 0, float>", "k_op FP32 tangent"),
            ("k_tau<6>", "k_tau"), ("k_gather<6, double>", "k_gather FP64")]
    lines = [
        "# Instruction issue of the element kernels, junction 1M tets (E = %d), K = 6" % E,
        "# Commands (repository root, one MI355X), one rocprofv3 run per counter pass:",
    ]
    for i, ctr in enumerate(ISSUE_PASSES):
        lines.append(f"#   rocprofv3 --pmc {ctr} --output-format csv -d rocprof_out/issue{'ABC'[i]} "
                     f"-o {'abc'[i]} -- python -u bench.py --probe --warmup 5")
    lines.append("#   python bench.py --summarize-issue <issueA csv> <issueB csv> <issueC csv>")
    lines.append("# The probe runs the benchmark's 5 warm-up Newton steps first (6 tau launches at the")
    lines.append("# states the timed steps see), then 3 FP64 and 3 FP32 tangent products.")
    lines.append("# Values are per dispatch (averaged over the probe's dispatches of the kernel);")
    lines.append("# 'per element' divides by E for every kernel (the gather runs one wave per node).")
    lines.append("# FP64 flops counted = 64 x SQ_INSTS_VALU_FLOPS_FP64 (flops per wave instruction) +")
    lines.append("# 512 x SQ_INSTS_VALU_MFMA_MOPS_F64; the rate divides by the same dispatches' cycles.")
    for pat, label in want:
        names = [k for k in tot if pat in k]
        if not names:
            raise SystemExit(f"{pat}: no dispatch in the counter files")
        k = names[0]
        nd = max(len(disp[(k, p)]) for p in csvs)
        c = {n: v / nd for n, v in tot[k].items()}
        cyc = c["GRBM_GUI_ACTIVE"] / 8.0
        simd = 1024.0
        # SQ_INSTS_VALU_FLOPS_FP64 counts the flops of each wave instruction
        # (gfx950 counter definition): x 64 lanes; MFMA MOPS count 512 flops
        f64c = 64.0 * c["SQ_INSTS_VALU_FLOPS_FP64"] + 512.0 * c["SQ_INSTS_VALU_MFMA_MOPS_F64"]
        lines += [
            "",
            f"[{label}]  ({nd} dispatches)",
            f"kernel_cycles = {cyc:.4g}   (= {cyc / 2.4e3:.1f} us at 2.4 GHz)",
            f"waves = {c['SQ_WAVES']:.0f}",
            f"valu_insts_per_element = {c['SQ_INSTS_VALU'] / E:.1f}",
            f"mfma_insts_per_element = {c['SQ_INSTS_MFMA'] / E:.2f}",
            f"lds_insts_per_element = {c['SQ_INSTS_LDS'] / E:.1f}",
            f"salu_insts_per_element = {c['SQ_INSTS_SALU'] / E:.1f}",
            f"vmem_rd_insts_per_element = {c['SQ_INSTS_VMEM_RD'] / E:.2f}",
            f"mfma_f64_flops_per_element = {c['SQ_INSTS_VALU_MFMA_MOPS_F64'] * 512 / E:.0f}",
            f"mfma_f32_flops_per_element = {c['SQ_INSTS_VALU_MFMA_MOPS_F32'] * 512 / E:.0f}",
            f"simd_frac_mfma_busy = {c['SQ_VALU_MFMA_BUSY_CYCLES'] / (cyc * simd):.3f}",
            f"simd_frac_valu_issue = {4.0 * c['SQ_ACTIVE_INST_VALU'] / (cyc * simd):.3f}",
            f"simd_frac_lds_active = {4.0 * c['SQ_ACTIVE_INST_LDS'] / (cyc * simd):.3f}",
            f"cu_frac_lds_bank_conflict = {c['SQ_LDS_BANK_CONFLICT'] / (cyc * 256.0):.3f}",
            f"wave_frac_waiting_on_counters = {c['SQ_WAIT_ANY'] / c['SQ_WAVE_CYCLES']:.3f}",
            f"wave_frac_waiting_to_issue = {c['SQ_WAIT_INST_ANY'] / c['SQ_WAVE_CYCLES']:.3f}",
            f"wave_frac_waiting_lds_issue = {c['SQ_WAIT_INST_LDS'] / c['SQ_WAVE_CYCLES']:.3f}",
            f"fp64_flops_counted_per_dispatch = {f64c:.6g}",
            f"fp64_tflops_counted = {f64c / (cyc / 2.4e9) / 1e12:.4g}",
            f"frac_fp64_peak_counted = {f64c / (cyc / 2.4e9) / 1e12 / FP64_PEAK_TFLOPS:.4f}",
        ]
    lines.append("")
    lines.append(f"kernel_source_hash = {kernel_source_hash()}")
    with open(ISSUE_FILE, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def batched(args):
    print(json.dumps(batched_run(args.batched, args.batch_concurrency, args.batch_graph)), flush=True)


def batched_run(N, concurrency=8, graph=False):
    """Batched solves: N inflow waveforms of uneven harmonic count on the
    Womersley pipe (R = 1, L = 4, 6,144 tets), K drawn from {3, 5, 7, 11},
    waveform Q(t)/Qbar = 1 + sum_k a k^-2 cos(k omega t + phi_k) with
    a ~ U[0.1, 1] and seeded phases, each solved to 1e-8 from the initial
    guess.  Runs them one at a time, then all through tsgls_solve_batch, and
    returns throughput and per-solve latency percentiles of both.  (On the
    200k-tet junction a solve to 1e-8 takes tens of thousands of products,
    so it is not a batch-latency workload.)"""
    import numpy as np
    import torch
    import paper_2311_09465_amd as T
    from workloads import womersley_problem, initial_guess
    from workloads.problems import inlet_waveforms
    from workloads.meshgen import pipe
    rng = np.random.default_rng(2311)
    mesh = pipe(4, 16)
    Ks = rng.choice([3, 5, 7, 11], size=N)
    amps = rng.uniform(0.1, 1.0, size=N)
    probs = [womersley_problem(K=int(Ks[i]), mesh=mesh,
                               waveform=inlet_waveforms(int(Ks[i]), 1000 + i, amps[i], n_inlets=1)[0])
             for i in range(N)]
    solvers = [T.Solver.from_problem(p, stream=torch.cuda.Stream()) for p in probs]
    opts = dict(rtol=1e-8, lin_rtol=0.05, restart=30, max_newton=40, gmres_graph=graph)
    # one short solve per K first (first-use setup of each kernel family)
    for K in sorted(set(int(k) for k in Ks)):
        i = int(np.argmax(Ks == K))
        y = torch.from_numpy(initial_guess(probs[i])).cuda()
        torch.cuda.synchronize()
        solvers[i].solve(y, **dict(opts, max_newton=1))
    torch.cuda.synchronize()

    def pct(x, q):
        return float(np.percentile(np.asarray(x), q))

    seq_lat, seq_ok, seq_it = [], 0, []
    t0 = time.perf_counter()
    for s, p in zip(solvers, probs):
        y = torch.from_numpy(initial_guess(p)).cuda()
        torch.cuda.synchronize()
        st = s.solve(y, **opts)
        seq_lat.append(time.perf_counter() - t0)
        seq_ok += st["status"] == 0
        seq_it.append(st["newton_iters"])
    seq_wall = time.perf_counter() - t0
    seq_own = np.diff([0.0] + seq_lat)
    ys = [torch.from_numpy(initial_guess(p)).cuda() for p in probs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, stats, fin = T.solve_batch(solvers, ys, max_concurrent=concurrency, **opts)
    bat_wall = time.perf_counter() - t0
    out = {
        "metric": "batched solves to 1e-8: throughput and per-solve latency",
        "n_solves": N, "n_gpus": 1, "data": "synthetic (seeded pipe inflow waveforms)",
        "config": dict(workload="womersley_6k_batched", n_tets=mesh.n_tets,
                       n_nodes=mesh.n_nodes, K_choices=[3, 5, 7, 11],
                       K_counts={int(k): int((Ks == k).sum()) for k in sorted(set(Ks.tolist()))},
                       restart=30, lin_rtol=0.05, concurrency=concurrency,
                       gmres_graph=bool(graph)),
        "sequential": dict(wall_s=round(seq_wall, 3), solves_per_s=round(N / seq_wall, 3),
                           own_p50_s=round(pct(seq_own, 50), 4), own_p99_s=round(pct(seq_own, 99), 4),
                           converged=int(seq_ok), newton_iters_mean=round(float(np.mean(seq_it)), 2)),
        "batched": dict(wall_s=round(bat_wall, 3), solves_per_s=round(N / bat_wall, 3),
                        latency_p50_s=round(pct(fin, 50), 4), latency_p99_s=round(pct(fin, 99), 4),
                        own_p50_s=round(pct([s_["seconds"] for s_ in stats], 50), 4),
                        own_p99_s=round(pct([s_["seconds"] for s_ in stats], 99), 4),
                        converged=int(sum(s_["status"] == 0 for s_ in stats)), status=rc),
        "throughput_gain": round(seq_wall / bat_wall, 3),
    }
    del solvers
    torch.cuda.empty_cache()
    out["lockstep"] = lockstep_run(probs, Ks, opts)
    out["lockstep"]["throughput_gain_vs_sequential"] = round(
        out["lockstep"]["solves_per_s"] / out["sequential"]["solves_per_s"], 3)
    return out


def lockstep_one_k(N, K):
    """N pipe waveforms (6,144 tets) of one harmonic count K, seeded as in
    batched_run, solved to 1e-8 as the segments of one context (no other
    leg: the workload of the lockstep kernel profile)."""
    import numpy as np
    import torch
    import paper_2311_09465_amd as T
    from workloads import womersley_problem, initial_guess
    from workloads.problems import inlet_waveforms
    from workloads.meshgen import pipe
    rng = np.random.default_rng(7)
    mesh = pipe(4, 16)
    amps = rng.uniform(0.1, 1.0, size=N)
    probs = [womersley_problem(K=K, mesh=mesh, waveform=inlet_waveforms(K, 500 + i, amps[i], n_inlets=1)[0])
             for i in range(N)]
    seg = T.SegmentSolver.from_problems(probs)
    y = torch.from_numpy(np.concatenate([initial_guess(p) for p in probs])).cuda()
    torch.cuda.synchronize()
    opts = dict(rtol=1e-8, lin_rtol=0.05, restart=30, max_newton=40)
    t0 = time.perf_counter()
    rc, stats, fin = seg.solve_segments(y, **opts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    seg.close()
    return dict(workload=f"womersley_6k_K{K}_lockstep{N}", n_solves=N, wall_s=round(wall, 3),
                solves_per_s=round(N / wall, 3), converged=int(sum(s_["status"] == 0 for s_ in stats)),
                products=int(sum(s_["matvecs"] for s_ in stats)),
                latency_p50_s=round(float(np.percentile(fin, 50)), 4),
                latency_p99_s=round(float(np.percentile(fin, 99)), 4), solver=opts)


def lockstep_run(probs, Ks, opts):
    """The same problems solved as segments: one context per harmonic count
    holding all of that count's waveforms (tsgls_solve_segments, graph-
    captured cycles of `restart` steps, restart <= 32), the four groups run
    concurrently from four host threads, each on its own stream.  Latency of
    a solve = time from the common start until its segment finished."""
    import threading
    import numpy as np
    import torch
    import paper_2311_09465_amd as T
    from workloads import initial_guess
    groups = {}
    for i, K in enumerate(Ks):
        groups.setdefault(int(K), []).append(i)
    so = dict(rtol=opts["rtol"], lin_rtol=opts["lin_rtol"], restart=opts["restart"],
              max_newton=opts["max_newton"])
    segs, ys = {}, {}
    for K, idx in groups.items():
        segs[K] = T.SegmentSolver.from_problems([probs[i] for i in idx], stream=torch.cuda.Stream())
        ys[K] = torch.from_numpy(np.concatenate([initial_guess(probs[i]) for i in idx])).cuda()
    # first use of each kernel family and of the graph capture, outside the timing
    for K in groups:
        y = ys[K].clone()
        torch.cuda.synchronize()
        segs[K].solve_segments(y, **dict(so, max_newton=1))
    torch.cuda.synchronize()
    res, errs = {}, []

    def run(K):
        try:
            res[K] = segs[K].solve_segments(ys[K], **so)
        except Exception as e:  # reported below
            errs.append(repr(e))

    t0 = time.perf_counter()
    th = [threading.Thread(target=run, args=(K,)) for K in groups]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if errs:
        raise RuntimeError("; ".join(errs))
    lat, conv, iters, group_wall = [], 0, [], {}
    for K, idx in groups.items():
        rc, stats, fin = res[K]
        lat += fin
        conv += sum(s_["status"] == 0 for s_ in stats)
        iters += [s_["newton_iters"] for s_ in stats]
        group_wall[K] = round(max(fin), 3)
    for s_ in segs.values():
        s_.close()
    N = len(probs)
    return dict(wall_s=round(wall, 3), solves_per_s=round(N / wall, 3),
                latency_p50_s=round(float(np.percentile(lat, 50)), 4),
                latency_p99_s=round(float(np.percentile(lat, 99)), 4),
                converged=int(conv), newton_iters_mean=round(float(np.mean(iters)), 2),
                group_wall_s=group_wall, restart=so["restart"], graph_cycles=True)


def learned(args):
    print(json.dumps(learned_run(args.learned, args.learned_test, args.learned_basis,
                                 args.learned_hidden, args.learned_steps, args.learned_precision)),
          flush=True)


def learned_run(ntr, nte, r, hidden=4, steps=3000, precision="bf16"):
    """Learned warm start on the pipe family (6,144 tets, K = 3; inflow
    waveform amplitude, phases, Re and Wo drawn per member): solves the
    training members (batched), builds the reduced basis, trains the
    network, then solves held-out members from the plain initial guess and
    from the prediction to the same absolute residual (1e-8 of the initial
    guess's).  Returns the measurements."""
    import numpy as np
    import torch
    import paper_2311_09465_amd as T
    from paper_2311_09465_amd.warmstart import WarmStart, fix_dirichlet
    from workloads import pipe_family, initial_guess
    probs, feats = pipe_family(ntr + nte, K=3, seed=11)
    opts = dict(lin_rtol=0.05, restart=30, max_newton=60)
    t0 = time.perf_counter()
    print(f"solving {ntr} training members", file=sys.stderr, flush=True)
    ys, rcs, chunk = [], [], 512     # contexts made and freed per chunk (device memory)
    for c0 in range(0, ntr, chunk):
        idx = range(c0, min(ntr, c0 + chunk))
        solvers = [T.Solver.from_problem(probs[i], stream=torch.cuda.Stream()) for i in idx]
        yc = [torch.from_numpy(initial_guess(probs[i])).cuda() for i in idx]
        torch.cuda.synchronize()
        rc, st, _ = T.solve_batch(solvers, yc, rtol=1e-9, max_concurrent=8, **opts)
        rcs.append(rc)
        ys += yc
        del solvers
        print(f"  {len(ys)} solved", file=sys.stderr, flush=True)
    rc = next((x for x in rcs if x != 0), 0)
    t_data = time.perf_counter() - t0
    print(f"training data in {t_data:.1f} s", file=sys.stderr, flush=True)
    Y = torch.stack([y.view(-1) for y in ys]).contiguous()
    del ys
    t0 = time.perf_counter()
    ws = WarmStart.fit(feats[:ntr], Y, r=r, n_hidden=hidden, steps=steps,
                       lr=1e-3, seed=1, precision=precision)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    rows = []
    for i in range(ntr, ntr + nte):
        p = probs[i]
        s = T.Solver.from_problem(p)
        y0 = torch.from_numpy(initial_guess(p)).cuda()
        r_cold = s.solve(y0.clone(), rtol=1.0, max_newton=0)["r0_norm"]
        yc = y0.clone()
        sc = s.solve(yc, rtol=1e-8, **opts)
        try:   # the Newton tangent from the plain initial guess, for comparison (bounded)
            scn = s.solve(y0.clone(), rtol=1e-8, jacobian="newton", **dict(opts, max_newton=30),
                          max_matvec=1000)
            cn = (scn["newton_iters"], scn["seconds"], scn["status"] == 0)
        except T.TsglsError:
            cn = (opts["max_newton"], float("nan"), False)
        torch.cuda.synchronize()
        a = time.perf_counter()
        yp = fix_dirichlet(ws.predict(feats[i:i + 1], [y0])[0], y0, p.dirichlet_nodes)
        torch.cuda.synchronize()
        t_pred = time.perf_counter() - a
        r_warm = s.solve(yp.clone(), rtol=1.0, max_newton=0)["r0_norm"]
        fallback = not r_warm < r_cold
        if fallback:
            yp, r_warm = y0.clone(), r_cold
        ypn = yp.clone()
        sw = s.solve(yp, rtol=1e-8 * r_cold / r_warm, **opts)
        # the prediction is close enough for the Newton tangent (tau frozen)
        swn = s.solve(ypn, rtol=1e-8 * r_cold / r_warm, jacobian="newton", **opts)
        # best the basis can do: the converged solution projected on it
        coef = T.rb_project(ws.Phi, yc.view(1, -1), ws.mean)[0].contiguous()
        ypr = torch.empty_like(yc)
        T.rb_expand(ws.Phi, coef, ws.mean, ypr.view(-1))
        ypr = fix_dirichlet(ypr, y0, p.dirichlet_nodes)
        r_proj = s.solve(ypr, rtol=1.0, max_newton=0)["r0_norm"]
        rows.append(dict(cold_it=sc["newton_iters"], warm_it=sw["newton_iters"], cold_s=sc["seconds"],
                         warm_s=sw["seconds"] + t_pred, ratio=r_warm / r_cold, proj=r_proj / r_cold,
                         ok=sc["status"] == 0 and sw["status"] == 0, fallback=fallback,
                         wn_it=swn["newton_iters"], wn_s=swn["seconds"] + t_pred,
                         wn_ok=swn["status"] == 0, cn_it=cn[0], cn_s=cn[1], cn_ok=cn[2]))
        print(f"member {i}: cold {sc['newton_iters']} (newton tangent {cn[0]}), warm {sw['newton_iters']}, "
              f"warm newton tangent {swn['newton_iters']}", file=sys.stderr, flush=True)

    def col(k):
        return np.array([row[k] for row in rows], dtype=float)

    out = {
        "metric": "learned warm start: Newton steps and time to 1e-8 vs the plain initial guess",
        "n_gpus": 1, "data": "synthetic (seeded pipe inflow waveforms, Re, Wo)",
        "config": dict(workload="womersley_6k_K3_family", n_tets=probs[0].mesh.n_tets, K=3,
                       n_train=ntr, n_test=nte, basis=int(ws.Phi.shape[0]), net=f"8-512x{hidden}-r tanh",
                       precision=("bf16 MFMA, FP32 master weights" if precision == "bf16"
                                  else "FP32 MFMA"), steps=steps),
        "train": dict(data_s=round(t_data, 3), all_converged=rc == 0, fit_s=round(t_fit, 3),
                      final_loss=ws.train_loss),
        "cold": dict(newton_mean=round(col("cold_it").mean(), 3), s_mean=round(col("cold_s").mean(), 4),
                     s_p50=round(float(np.median(col("cold_s"))), 4)),
        "warm": dict(newton_mean=round(col("warm_it").mean(), 3), s_mean=round(col("warm_s").mean(), 4),
                     s_p50=round(float(np.median(col("warm_s"))), 4),
                     residual_ratio_p50=float("%.3e" % np.median(col("ratio"))),
                     fallbacks=int(col("fallback").sum())),
        "cold_newton_tangent": dict(newton_mean=round(col("cn_it").mean(), 3),
                                    s_mean=round(float(np.nanmean(col("cn_s"))), 4),
                                    converged=int(col("cn_ok").sum())),
        "warm_newton_tangent": dict(newton_mean=round(col("wn_it").mean(), 3),
                                    s_mean=round(col("wn_s").mean(), 4),
                                    converged=int(col("wn_ok").sum())),
        "basis_projection_residual_ratio_p50": float("%.3e" % np.median(col("proj"))),
        "all_converged": bool(all(row["ok"] for row in rows)),
        "speedup_time_to_1e8": round(col("cold_s").mean() / col("warm_s").mean(), 3),
        "speedup_time_to_1e8_warm_newton": round(col("cold_s").mean() / col("wn_s").mean(), 3),
    }
    return out


JUNCTION_SOLVE = dict(rtol=1e-8, lin_rtol=0.1, restart=100, max_newton=150, max_matvec=10000,
                      jacobian="newton", dt_pseudo=0.1, dt_schedule="ser", dt_max=2.0)
# K = 6: unbounded step, GMRES(60), 3,000 products per linear solve (a short
# solve halves the next step)
JUNCTION_SOLVE_K6 = dict(JUNCTION_SOLVE, max_newton=250, max_matvec=3000, dt_max=0.0, restart=60)


def junction_time_to_1e8():
    """Time to 1e-8 on the 200k-tet junction (h = 0.081, K = 3, Re = 100,
    Wo = 10) from the initial guess: pseudo-time stepping with one Newton
    iteration per step (Newton tangent, tau frozen), switched-evolution step
    size from 0.1 bounded by 2, GMRES(100) to 0.1; FP64 tangent, FP32
    tangent and FP32 tangent with tau in bf16 (FP64 residual and Krylov).
    Then K = 6 with the FP32 tangent, the step unbounded, GMRES(60) and
    3,000 products per linear solve.  Returns the summary and, when the FP64 solve
    converged, (problem, its converged state, flow summary) for the tracer
    leg, else None."""
    import torch
    import paper_2311_09465_amd as T
    from workloads import junction_problem, initial_guess
    prob = junction_problem(h=0.081, K=3, Re=100.0)
    s = T.Solver.from_problem(prob)
    out = dict(workload="junction_200k_K3_Re100", n_tets=prob.mesh.n_tets, n_nodes=prob.mesh.n_nodes,
               solver={k: v for k, v in JUNCTION_SOLVE.items()})
    flow = None
    for prec in ("f64", "f32", "bf16"):
        y = torch.from_numpy(initial_guess(prob)).cuda()
        torch.cuda.synchronize()
        st = s.solve(y, tangent_precision=prec, **JUNCTION_SOLVE)
        if prec == "f64" and st["status"] == 0:
            flow = (prob, y, dict(status=st["status"], rel_residual=st["rel_residual"],
                                  seconds=round(st["seconds"], 3), tangent="f64"))
        out[prec] = dict(seconds=round(st["seconds"], 3), status="converged" if st["status"] == 0
                         else "not converged", newton_iters=st["newton_iters"], matvecs=st["matvecs"],
                         rel_residual=float("%.3e" % st["rel_residual"]), rejected=st["rejected"])
        print(f"junction 200k time to 1e-8 ({prec}): {out[prec]}", file=sys.stderr, flush=True)
    out["f32_speedup"] = round(out["f64"]["seconds"] / out["f32"]["seconds"], 3)
    out["bf16_speedup"] = round(out["f64"]["seconds"] / out["bf16"]["seconds"], 3)
    s.close()
    del s
    torch.cuda.empty_cache()
    prob = junction_problem(h=0.081, K=6, Re=100.0)
    s = T.Solver.from_problem(prob)
    y = torch.from_numpy(initial_guess(prob)).cuda()
    torch.cuda.synchronize()
    st = s.solve(y, tangent_precision="f32", **JUNCTION_SOLVE_K6)
    out["K6_f32"] = dict(workload="junction_200k_K6_Re100", solver=dict(JUNCTION_SOLVE_K6),
                         seconds=round(st["seconds"], 3),
                         status="converged" if st["status"] == 0 else "not converged",
                         newton_iters=st["newton_iters"], matvecs=st["matvecs"],
                         rel_residual=float("%.3e" % st["rel_residual"]), rejected=st["rejected"],
                         short_linear_solves=st["lin_unconverged"])
    print(f"junction 200k K=6 time to 1e-8 (f32): {out['K6_f32']}", file=sys.stderr, flush=True)
    s.close()
    return out, flow


def mode_sweep_200k(ks=(3, 7, 15, 31), reps=20):
    """Per-K cost on the 200k-tet junction (h = 0.081, Re = 500, Wo = 10) at
    a seeded state (initial guess + 0.05 noise): linearize (tau at every
    point, residual) and the tangent product in FP64 and with the FP32
    element operator, back to back after warm-ups, with the product rate in
    the metric's unit and the FP32 product's max-norm difference from the
    FP64 one relative to its largest entry."""
    import numpy as np
    import torch
    import paper_2311_09465_amd as T
    from workloads import junction_problem, initial_guess
    out = {}
    for K in ks:
        prob = junction_problem(h=0.081, K=K, Re=500.0, Wo=10.0, seed=1)
        rng = np.random.default_rng(100 + K)
        y0 = initial_guess(prob)
        noise = 0.05 * rng.standard_normal(y0.shape)
        noise[..., 1] = 0.0
        noise[prob.dirichlet_nodes, :3] = 0.0
        y = torch.from_numpy(y0 + noise).cuda()
        v = torch.from_numpy(rng.standard_normal(y0.shape)).cuda()
        s = T.Solver.from_problem(prob)
        r = torch.zeros_like(y)
        o64, o32 = torch.zeros_like(y), torch.zeros_like(y)

        def timed(call, n):
            call()
            torch.cuda.synchronize()
            a = time.perf_counter()
            for _ in range(n):
                call()
            torch.cuda.synchronize()
            return (time.perf_counter() - a) / n * 1e3

        lin_ms = timed(lambda: s.linearize(y, r), 3)
        s.jv(v, o32, "picard", precision="f32")
        jv64 = timed(lambda: s.jv(v, o64, "picard"), reps)
        jv32 = timed(lambda: s.jv(v, o32, "picard", precision="f32"), reps)
        torch.cuda.synchronize()
        diff = float((o32 - o64).abs().max() / o64.abs().max())
        dof = prob.mesh.n_nodes * 4 * (2 * K + 1)
        out[f"K{K}"] = dict(n=2 * K + 1, M=3 * K + 1, linearize_ms=round(lin_ms, 3),
                            jv_f64_ms=round(jv64, 3), jv_f32_ms=round(jv32, 3),
                            jv_f64_gdof_modes_s=round(dof / jv64 / 1e6, 4),
                            jv_f32_gdof_modes_s=round(dof / jv32 / 1e6, 4),
                            f32_vs_f64_rel_maxdiff=float("%.2e" % diff))
        print(f"mode sweep K={K}: {out[f'K{K}']}", file=sys.stderr, flush=True)
        s.close()
        del s, y, v, r, o64, o32
        torch.cuda.empty_cache()
    return dict(workload="junction_200k", n_tets=prob.mesh.n_tets, n_nodes=prob.mesh.n_nodes, **out)


def junction_re500_attempt(prob, steps=25):
    """The headline junction (Re = 500) in pseudo-time with the Newton
    tangent and a fixed step of 0.3, bounded to `steps` pseudo-time steps of
    at most 300 products: the relative residual does not settle (no attractor
    of the pseudo-time iteration), so only its trace is reported.  (With the
    adaptive schedule every step here is cut short by the product budget, so
    the step keeps halving and the trace stalls near 0.5.)"""
    import torch
    import paper_2311_09465_amd as T
    from workloads import initial_guess
    s = T.Solver.from_problem(prob)
    y = torch.from_numpy(initial_guess(prob)).cuda()
    torch.cuda.synchronize()
    st = s.solve(y, **dict(JUNCTION_SOLVE, max_newton=steps, max_matvec=300, dt_pseudo=0.3,
                           dt_schedule="fixed", dt_max=0.0))
    h = st["history"]
    s.close()
    return dict(workload="junction_1M_K6_Re500", schedule="fixed dt 0.3, Newton tangent, 300 products",
                pseudo_time_steps=st["newton_iters"],
                matvecs=st["matvecs"], seconds=round(st["seconds"], 3),
                rel_residual_min=float("%.3e" % min(h)), rel_residual_last=float("%.3e" % h[-1]),
                history=[float("%.2e" % x) for x in h])


def dt_sweep(args):
    """Pseudo-time step sweep: Newton-GMRES with the mass shift 1.5 rho/dt in
    the tangent (dt = inf: plain Newton) on the pipe (6,144 tets, K = 3,
    Re 100) and on the 200k-tet junction (K = 3, Re 100); relative residual
    history per dt.  Prints one JSON line."""
    import numpy as np
    import torch
    import paper_2311_09465_amd as T
    from workloads import womersley_problem, junction_problem, initial_guess
    dts = [0.0, 1.0, 0.3, 0.1, 0.03]
    cases = [("womersley_6k_K3", womersley_problem(4, 16, K=3), 30),
             ("junction_200k_K3_Re100", junction_problem(h=0.081, K=3, Re=100.0, seed=1), args.dt_sweep)]
    out = {"metric": "pseudo-time step sweep: relative residual after Newton steps",
           "n_gpus": 1, "data": "synthetic", "cases": {}}
    for name, prob, nmax in cases:
        s = T.Solver.from_problem(prob)
        res = []
        for dt in dts:
            y = torch.from_numpy(initial_guess(prob)).cuda()
            torch.cuda.synchronize()
            try:
                st = s.solve(y, rtol=1e-8, lin_rtol=0.05, restart=30, max_newton=nmax, max_matvec=3000,
                             dt_pseudo=dt)
                res.append(dict(dt="inf" if dt == 0 else dt, converged=st["status"] == 0,
                                newton=st["newton_iters"], matvecs=st["matvecs"],
                                seconds=round(st["seconds"], 3), final=float("%.3e" % st["rel_residual"]),
                                history=[float("%.2e" % h) for h in st["history"]]))
            except T.TsglsError as e:
                res.append(dict(dt="inf" if dt == 0 else dt, error=str(e)))
            print(f"{name} dt={dt}: {res[-1].get('final', res[-1].get('error'))}", file=sys.stderr, flush=True)
        out["cases"][name] = dict(n_tets=prob.mesh.n_tets, max_newton=nmax, runs=res)
        del s
    print(json.dumps(out), flush=True)


def tracer(args):
    """Tracer (convection-diffusion) carried by the converged pipe flow
    (6,144 tets, K = 3, Re 100, Wo 5): phi = 1 at the inlet, 0 at the outlet,
    GLS against Galerkin (tau = 0) for several diffusivities; unpreconditioned
    GMRES to 1e-8, products and time, and the range of phi over the nodes at
    3K+1 instants of the period (bounded by [0, 1] in the exact solution).
    Prints one JSON line."""
    import numpy as np
    import torch
    import paper_2311_09465_amd as T
    from workloads import womersley_problem, initial_guess
    prob = womersley_problem(4, 16, K=3)
    K = 3
    ns = T.Solver.from_problem(prob)
    yv = torch.from_numpy(initial_guess(prob)).cuda()
    ns.solve(yv, rtol=1e-8, restart=30)

    def nodes(t):
        return np.unique(np.asarray(t).ravel())

    wall = nodes(prob.mesh.faces["wall"])
    dn = np.setdiff1d(np.union1d(nodes(prob.mesh.faces["inlet"]), nodes(prob.mesh.faces["outlet"])), wall)
    inlet = np.intersect1d(dn, nodes(prob.mesh.faces["inlet"]))
    M = 3 * K + 1
    t = 2 * np.pi * np.arange(M) / M
    runs = []
    for kappa in (0.02, 0.005, 0.001):
        for stab in (True, False):
            s = T.Solver(prob.mesh.xyz, prob.mesh.tets, K, prob.rho, prob.mu, prob.omega)
            s.set_dirichlet(dn.astype(np.int32))
            s.set_tracer(yv, kappa, stab)
            y0 = np.zeros((prob.mesh.n_nodes, 4, 2 * K + 2))
            y0[inlet, 0, 0] = 1.0
            y = torch.from_numpy(y0).cuda()
            st = s.solve(y, rtol=1e-8, lin_rtol=1e-8, restart=100, max_newton=1, max_matvec=20000)
            ph = y.cpu().numpy()[:, 0]
            c = ph[:, 0::2] + 1j * ph[:, 1::2]
            c[:, 0] = ph[:, 0]
            vals = c[:, :1].real + 2 * np.real(sum(c[:, k:k + 1] * np.exp(1j * k * t)[None, :]
                                                   for k in range(1, K + 1)))
            runs.append(dict(kappa=kappa, method="GLS" if stab else "Galerkin",
                             converged=st["status"] == 0, gmres_products=st["matvecs"],
                             rel_residual=float("%.2e" % st["rel_residual"]),
                             seconds=round(st["seconds"], 3),
                             phi_min=float("%.3e" % vals.min()), phi_max=float("%.3e" % vals.max())))
            print(runs[-1], file=sys.stderr, flush=True)
            del s
    # Backflow: a reversing inflow Q(t) = Qbar (1 + 1.6 sin wt) makes fluid re-enter through the
    # outlet for part of the period; the outlet is a natural boundary of the tracer
    # (phi = 1 + 0.5 cos wt at the inlet only), with the backflow term at beta = 0.5 and without
    # it (beta = 0), for two diffusivities.
    pb = womersley_problem(4, 16, K=3, amp=1.6)
    nsb = T.Solver.from_problem(pb)
    yb = torch.from_numpy(initial_guess(pb)).cuda()
    stb = nsb.solve(yb, rtol=1e-8, restart=30, max_newton=60)
    outl = nodes(pb.mesh.faces["outlet"])
    ub = yb.cpu().numpy()[outl, 2]                       # axial velocity = u.n on the outlet
    cu = ub[:, 0::2] + 1j * ub[:, 1::2]
    cu[:, 0] = ub[:, 0]
    uz = cu[:, :1].real + 2 * np.real(sum(cu[:, k:k + 1] * np.exp(1j * k * t)[None, :]
                                          for k in range(1, K + 1)))
    dnb = np.setdiff1d(nodes(pb.mesh.faces["inlet"]), nodes(pb.mesh.faces["wall"]))
    back = []
    for kappa, beta in ((0.005, 0.5), (0.005, 0.0), (0.001, 0.5), (0.001, 0.0)):
        s = T.Solver(pb.mesh.xyz, pb.mesh.tets, K, pb.rho, pb.mu, pb.omega, backflow_beta=beta)
        s.set_dirichlet(dnb.astype(np.int32))
        s.set_neumann(np.asarray(pb.mesh.faces["outlet"], dtype=np.int32))
        s.set_tracer(yb, kappa, True)
        y0 = np.zeros((pb.mesh.n_nodes, 4, 2 * K + 2))
        y0[dnb, 0, 0] = 1.0
        y0[dnb, 0, 2] = 0.25                            # Re c_1: 0.5 cos wt
        y = torch.from_numpy(y0).cuda()
        st = s.solve(y, rtol=1e-8, lin_rtol=1e-8, restart=100, max_newton=1, max_matvec=20000)
        ph = y.cpu().numpy()[:, 0]
        c = ph[:, 0::2] + 1j * ph[:, 1::2]
        c[:, 0] = ph[:, 0]
        vals = c[:, :1].real + 2 * np.real(sum(c[:, k:k + 1] * np.exp(1j * k * t)[None, :]
                                               for k in range(1, K + 1)))
        back.append(dict(kappa=kappa, beta=beta, converged=st["status"] == 0, gmres_products=st["matvecs"],
                         rel_residual=float("%.2e" % st["rel_residual"]),
                         phi_min=float("%.3e" % vals.min()), phi_max=float("%.3e" % vals.max())))
        print(back[-1], file=sys.stderr, flush=True)
        del s
    print(json.dumps({"metric": "tracer: GLS vs Galerkin, GMRES products to 1e-8 and range of phi",
                      "n_gpus": 1, "data": "synthetic (converged pipe flow)",
                      "config": dict(workload="womersley_6k_K3_tracer", n_tets=prob.mesh.n_tets, K=K,
                                     restart=100, preconditioner="none"),
                      "runs": runs,
                      "backflow": dict(flow="Q(t) = Qbar (1 + 1.6 sin wt)", method="GLS",
                                       inlet_phi="1 + 0.5 cos wt",
                                       ns_converged=stb["status"] == 0,
                                       outlet_min_axial_velocity=float("%.3e" % uz.min()),
                                       runs=back)}), flush=True)


def junction_solve(args):
    """One leg of time_to_1e8_junction alone: the 200k-tet junction (h =
    0.081, K = 3, Re = 100, Wo = 10) from the initial guess to 1e-8 with the
    same pseudo-time settings and the given tangent precision, printing each
    pseudo-time step (so that a kernel trace of the whole solve can be taken).
    Prints one JSON line."""
    import torch
    import paper_2311_09465_amd as T
    from workloads import junction_problem, initial_guess
    prob = junction_problem(h=0.081, K=3, Re=100.0)
    s = T.Solver.from_problem(prob)
    y = torch.from_numpy(initial_guess(prob)).cuda()
    torch.cuda.synchronize()
    st = s.solve(y, tangent_precision=args.junction_solve, verbose=True, **JUNCTION_SOLVE)
    print(json.dumps(dict(workload="junction_200k_K3_Re100", tangent=args.junction_solve,
                          solver=dict(JUNCTION_SOLVE), seconds=round(st["seconds"], 3),
                          status="converged" if st["status"] == 0 else "not converged",
                          newton_iters=st["newton_iters"], matvecs=st["matvecs"],
                          rel_residual=float("%.3e" % st["rel_residual"]))), flush=True)


def tracer_junction(args):
    """Tracer on the 200k-tet junction (h = 0.081, K = 3, Re = 100, Wo = 10)
    carried by its converged periodic flow (pseudo-time solve to 1e-8):
    phi = 1 on the larger inlet, 0 on the smaller one, walls natural, the
    outlets either zero Dirichlet (the paper's case: a rapid jump) or natural
    with the backflow term (beta = 0.5); GLS against Galerkin
    (tau = 0) for two diffusivities, unpreconditioned GMRES(100) to 1e-8
    (at most 20,000 products); products, time and the range of phi over the
    nodes at 3K+1 instants (within [0, 1] for the exact solution).  Prints
    one JSON line."""
    import torch
    import paper_2311_09465_amd as T
    from workloads import junction_problem, initial_guess
    prob = junction_problem(h=0.081, K=3, Re=100.0)
    ns = T.Solver.from_problem(prob)
    yv = torch.from_numpy(initial_guess(prob)).cuda()
    stn = ns.solve(yv, tangent_precision="f32", **JUNCTION_SOLVE)
    print(f"flow: {stn['status']} {stn['rel_residual']:.2e} {stn['seconds']:.1f}s", file=sys.stderr, flush=True)
    flow = dict(status=stn["status"], rel_residual=stn["rel_residual"], seconds=round(stn["seconds"], 3))
    print(json.dumps(tracer_junction_run(prob, yv, flow)), flush=True)


def tracer_junction_run(prob, yv, flow, outlet_cases=("dirichlet", "natural")):
    """The tracer runs of tracer_junction on the converged flow yv of prob."""
    import numpy as np
    import torch
    import paper_2311_09465_amd as T
    K = prob.K

    def nodes(t):
        return np.unique(np.asarray(t).ravel())

    wall = nodes(prob.mesh.faces["wall"])
    in1 = np.setdiff1d(nodes(prob.mesh.faces["in1"]), wall)
    in2 = np.setdiff1d(nodes(prob.mesh.faces["in2"]), wall)
    outl = np.setdiff1d(nodes(prob.neumann_tris), wall)
    M = 3 * K + 1
    t = 2 * np.pi * np.arange(M) / M
    runs = []
    # outlets: zero Dirichlet (the paper's test of a rapid jump) or natural with the backflow term
    for outlets in outlet_cases:
      for kappa in (0.005, 0.001):
        for stab in (True, False):
            s = T.Solver(prob.mesh.xyz, prob.mesh.tets, K, prob.rho, prob.mu, prob.omega,
                         backflow_beta=0.5)
            if outlets == "dirichlet":
                s.set_dirichlet(np.union1d(np.union1d(in1, in2), outl).astype(np.int32))
            else:
                s.set_dirichlet(np.union1d(in1, in2).astype(np.int32))
                s.set_neumann(prob.neumann_tris)
            s.set_tracer(yv, kappa, stab)
            y0 = np.zeros((prob.mesh.n_nodes, 4, 2 * K + 2))
            y0[in1, 0, 0] = 1.0
            y = torch.from_numpy(y0).cuda()
            st = s.solve(y, rtol=1e-8, lin_rtol=1e-8, restart=100, max_newton=1, max_matvec=20000)
            ph = y.cpu().numpy()[:, 0]
            c = ph[:, 0::2] + 1j * ph[:, 1::2]
            c[:, 0] = ph[:, 0]
            vals = c[:, :1].real + 2 * np.real(sum(c[:, k:k + 1] * np.exp(1j * k * t)[None, :]
                                                   for k in range(1, K + 1)))
            runs.append(dict(outlets=outlets, kappa=kappa, method="GLS" if stab else "Galerkin",
                             converged=st["status"] == 0, gmres_products=st["matvecs"],
                             rel_residual=float("%.2e" % st["rel_residual"]),
                             seconds=round(st["seconds"], 3),
                             phi_min=float("%.3e" % vals.min()), phi_max=float("%.3e" % vals.max())))
            print(runs[-1], file=sys.stderr, flush=True)
            s.close()
    return {"metric": "tracer on the junction: GLS vs Galerkin, GMRES products to 1e-8 and range of phi",
            "n_gpus": 1, "data": "synthetic (converged junction flow, Re 100)",
            "config": dict(workload="junction_200k_K3_Re100_tracer", n_tets=prob.mesh.n_tets,
                           K=K, restart=100, preconditioner="none", backflow_beta=0.5),
            "flow": flow, "runs": runs}


def tau_entry(prof, K, E, args):
    """tau's launch time over the timed steps and its FP64 rate by the
    60 n^3 per point model; beside it the counted rate (VALU + MFMA flops
    over the same dispatches' cycles, from the committed counter summary of
    the probe at the warm-up states) when that summary matches the sources."""
    ms = prof["tau"][1] / max(prof["tau"][0], 1)
    model = 60.0 * (2 * K + 1) ** 3 * 4 * E
    out = dict(ms_per_launch=round(ms, 3), tflops_model=round(model / (ms / 1e3) / 1e12, 3),
               frac_fp64_peak_model=round(model / (ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS, 4))
    cf = read_tau_counted() if (args.workload == "junction_1M_K6" and args.jacobian == "picard") else None
    out["counted"] = None if cf is None else dict(
        cf, source="profiles/k_op_junction_1M_K6_issue.txt (probe at the warm-up states)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="junction_1M_K6")
    ap.add_argument("--jv-per-step", type=int, default=30)
    ap.add_argument("--jacobian", default="picard")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-solves", action="store_true",
                    help="skip the solve measurements (junction time to 1e-8, batched, learned)")
    ap.add_argument("--probe", action="store_true",
                    help="counter-collection workload (linearize, 3 tangent products, a 512 MiB copy)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic summary under profiles/ from two rocprofv3 --pmc CSVs")
    ap.add_argument("--summarize-issue", nargs=3, metavar=("A_CSV", "B_CSV", "C_CSV"),
                    help="write the instruction-issue summary under profiles/ from three rocprofv3 "
                         "--pmc CSVs of the probe")
    ap.add_argument("--batched", type=int, default=0, metavar="N",
                    help="batched-solve measurement: N inflow waveforms on the 6k-tet pipe")
    ap.add_argument("--batch-concurrency", type=int, default=8)
    ap.add_argument("--batch-graph", action="store_true",
                    help="batched solves with graph-captured GMRES cycles")
    ap.add_argument("--lockstep", type=int, default=0, metavar="N",
                    help="lockstep measurement only: N pipe waveforms of one harmonic count "
                         "(--lockstep-k) as the segments of one context")
    ap.add_argument("--lockstep-k", type=int, default=7)
    ap.add_argument("--dt-sweep", type=int, default=0, metavar="MAX_NEWTON",
                    help="pseudo-time step sweep (junction runs MAX_NEWTON Newton steps)")
    ap.add_argument("--tracer", action="store_true",
                    help="tracer equation: GLS against Galerkin on the pipe flow")
    ap.add_argument("--tracer-junction", action="store_true",
                    help="tracer equation: GLS against Galerkin on the 200k junction flow")
    ap.add_argument("--junction-solve", default=None, choices=["f64", "f32", "bf16"],
                    help="one solve of the 200k junction to 1e-8 (K = 3) with this tangent, steps printed")
    ap.add_argument("--learned", type=int, default=0, metavar="N_TRAIN",
                    help="learned warm-start measurement with N_TRAIN training solves")
    ap.add_argument("--learned-test", type=int, default=32)
    ap.add_argument("--learned-basis", type=int, default=64)
    ap.add_argument("--learned-steps", type=int, default=3000)
    ap.add_argument("--learned-hidden", type=int, default=4, help="hidden layers of width 512")
    ap.add_argument("--learned-precision", default="bf16", choices=["bf16", "f32"])
    args = ap.parse_args()
    if args.summarize_issue:
        summarize_issue(args.summarize_issue)
        return
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc,
                      "rocprofv3 --pmc {counter} --output-format csv -d rocprof_out/{d} -o p -- "
                      "python -u bench.py --probe --warmup 5")
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; multi-GPU runs are not implemented "
                          "(mesh-partition sharding is described in the design notes)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2311_09465_amd as T
    from workloads import initial_guess

    torch.cuda.set_device(0)
    if args.probe:
        probe(args)
        return
    if args.batched:
        batched(args)
        return
    if args.lockstep:
        print(json.dumps(lockstep_one_k(args.lockstep, args.lockstep_k)), flush=True)
        return
    if args.learned:
        learned(args)
        return
    if args.dt_sweep:
        dt_sweep(args)
        return
    if args.tracer:
        tracer(args)
        return
    if args.tracer_junction:
        tracer_junction(args)
        return
    if args.junction_solve:
        junction_solve(args)
        return
    prob, cfg = _workload(args.workload)
    s = T.Solver.from_problem(prob)
    info = s.info()
    K, E, nn = prob.K, prob.mesh.n_tets, prob.mesh.n_nodes
    dof = nn * 4 * (2 * K + 1)
    y = torch.from_numpy(initial_guess(prob)).cuda()
    m = args.jv_per_step
    step_kw = dict(rtol=1e-300, lin_rtol=1e-300, restart=m, max_matvec=m, jacobian=args.jacobian)
    if args.warmup > 0:
        s.solve(y, max_newton=args.warmup, **step_kw)
    torch.cuda.synchronize()
    y_start = y.clone()   # the mixed-precision run below starts from the same state
    s.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.solve(y, max_newton=args.steps, **step_kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {k: s.profile_get(k) for k in s.PROF}
    s.profile(False)
    secs = t1 - t0
    value = args.steps * m * dof / secs / 1e9

    # dominant kernel: the element kernel of the tangent products (one launch
    # over all elements per product)
    launches, tot_ms = prof["elem_tangent"]
    avg_launch_s = tot_ms / max(launches, 1) / 1e3
    fl = jv_flops_per_element(K, args.jacobian) * E
    achieved = fl / avg_launch_s / 1e12
    tr = read_traffic() if (args.workload == "junction_1M_K6" and args.jacobian == "picard") else None
    roofline = dict(bound="alu", achieved=round(achieved, 3), peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / FP64_PEAK_TFLOPS, 4),
                    traffic=None if tr is None else round(tr["bytes_per_launch"]),
                    kernel="k_op<K,0> (tangent product element operator)",
                    avg_launch_us=round(avg_launch_s * 1e6, 2), launches=launches,
                    elements_per_launch=E,
                    flops_per_element=jv_flops_per_element(K, args.jacobian),
                    algorithmic_bytes_per_launch=round(jv_bytes(K, E, nn, args.jacobian)),
                    hbm_gbs_algorithmic=round(jv_bytes(K, E, nn, args.jacobian) / avg_launch_s / 1e9, 1))
    roofline["hbm_frac_algorithmic"] = round(jv_bytes(K, E, nn, args.jacobian) / avg_launch_s / 1e9
                                             / HBM_PEAK_GBS, 4)
    if tr is not None:
        roofline["hbm_gbs_measured"] = round(tr["bytes_per_launch"] / avg_launch_s / 1e9, 1)
        roofline["hbm_frac_measured"] = round(tr["bytes_per_launch"] / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4)
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "GDOF-modes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(secs / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded junction mesh and inflow waveforms)",
        "config": dict(cfg, n_tets=E, n_nodes=nn, jv_per_step=m, tangent=args.jacobian),
        "roofline": roofline,
        "breakdown_ms_per_step": {k: round(v[1] / args.steps, 3) for k, v in prof.items()},
        # tau: one launch per Newton step over 4 E points; model ~60 n^3 FP64 flops per point
        # (S, the Jacobi sweeps and Q^T Q), against the FP64 peak
        "tau": tau_entry(prof, K, E, args),
        "newton_rel_residual_after": st["rel_residual"],
    }
    if not args.no_extras:
        # pure tangent-product rate, back to back at the current linearization
        v = torch.randn_like(y)
        o = torch.zeros_like(y)
        for _ in range(5):
            s.jv(v, o, args.jacobian)
        torch.cuda.synchronize()
        reps = 50
        a = time.perf_counter()
        for _ in range(reps):
            s.jv(v, o, args.jacobian)
        torch.cuda.synchronize()
        jv_ms = (time.perf_counter() - a) / reps * 1e3
        out["jv_ms"] = round(jv_ms, 3)
        out["jv_only_gdof_modes_s"] = round(dof / jv_ms / 1e6, 4)
        # linearize (nodal samples, tau, face |A_n|_-, residual with z stored)
        # and the residual alone, in the same unit, 10 calls each after one
        r = torch.zeros_like(y)
        for name, call in (("linearize", lambda: s.linearize(y, r)), ("residual", lambda: s.residual(y, r))):
            call()
            torch.cuda.synchronize()
            a = time.perf_counter()
            for _ in range(10):
                call()
            torch.cuda.synchronize()
            t_ms = (time.perf_counter() - a) / 10 * 1e3
            out[f"{name}_ms"] = round(t_ms, 3)
            out[f"{name}_gdof_modes_s"] = round(dof / t_ms / 1e6, 4)
        s.linearize(y)   # the state the products below were measured at
        # mixed precision: the same steps, from the same state, with the FP32
        # element operator in the tangent (residual, tau, diagonal and Krylov
        # stay FP64), then the same with tau in bf16; one product of each kind
        # first allocates its copies
        def lower_precision(prec):
            s.jv(v, o, args.jacobian, precision=prec)
            y.copy_(y_start)
            torch.cuda.synchronize()
            s.profile(True)
            torch.cuda.synchronize()
            a = time.perf_counter()
            s.solve(y, max_newton=args.steps, tangent_precision=prec, **step_kw)
            torch.cuda.synchronize()
            secs_p = time.perf_counter() - a
            prof_p = {k: s.profile_get(k) for k in s.PROF}
            s.profile(False)
            lp, tp = prof_p["elem_tangent"]
            avg_p = tp / max(lp, 1) / 1e3
            s.jv(v, o, args.jacobian, precision=prec)
            torch.cuda.synchronize()
            a = time.perf_counter()
            for _ in range(reps):
                s.jv(v, o, args.jacobian, precision=prec)
            torch.cuda.synchronize()
            jv_p = (time.perf_counter() - a) / reps * 1e3
            tau_word = 2 if prec == "bf16" else 4
            n_, P_ = 2 * K + 1, (2 * K + 1) * (2 * K + 2) // 2
            alg = jv_bytes(K, E, nn, args.jacobian, word=4) - E * 4.0 * (4 - tau_word) * P_
            res = dict(
                value=round(args.steps * m * dof / secs_p / 1e9, 4),
                ms_per_step=round(secs_p / args.steps * 1e3, 3),
                breakdown_ms_per_step={k: round(v_[1] / args.steps, 3) for k, v_ in prof_p.items()},
                elem_tangent_avg_launch_us=round(avg_p * 1e6, 2),
                elem_tangent_tflops_fp32=round(fl / avg_p / 1e12, 3),
                elem_tangent_algorithmic_bytes=round(alg),
                elem_tangent_hbm_frac_algorithmic=round(alg / avg_p / 1e9 / HBM_PEAK_GBS, 4),
                jv_ms=round(jv_p, 3))
            return res

        out["mixed_f32_tangent"] = lower_precision("f32")
        out["mixed_f32_tangent"]["elem_tangent_traffic"] = None if tr is None else round(
            tr["f32_bytes_per_launch"])
        out["mixed_f32_tangent"]["elem_tangent_hbm_frac_measured"] = None if tr is None else round(
            tr["f32_bytes_per_launch"] / (out["mixed_f32_tangent"]["elem_tangent_avg_launch_us"] / 1e6)
            / 1e9 / HBM_PEAK_GBS, 4)
        out["bf16_tau_tangent"] = lower_precision("bf16")
        # time to 1e-8 on the small Womersley case (full solve, FP64, Picard)
        del s
        torch.cuda.empty_cache()
        pw, _ = _workload("womersley_6k_K3")
        sw = T.Solver.from_problem(pw)
        yw = torch.from_numpy(initial_guess(pw)).cuda()
        stw = sw.solve(yw, rtol=1e-8, lin_rtol=0.05, restart=100, max_newton=60)
        out["time_to_1e8_womersley_6k_K3_s"] = round(stw["seconds"], 4)
        out["time_to_1e8_womersley_6k_K3_newton_iters"] = stw["newton_iters"]
        out["time_to_1e8_womersley_6k_K3_matvecs"] = stw["matvecs"]
        yw = torch.from_numpy(initial_guess(pw)).cuda()
        stw = sw.solve(yw, rtol=1e-8, lin_rtol=0.05, restart=100, max_newton=60,
                       tangent_precision="f32")
        out["mixed_f32_tangent"].update(
            time_to_1e8_womersley_6k_K3_s=round(stw["seconds"], 4),
            time_to_1e8_womersley_6k_K3_newton_iters=stw["newton_iters"],
            time_to_1e8_womersley_6k_K3_matvecs=stw["matvecs"],
            time_to_1e8_womersley_6k_K3_status=stw["status"])
        del sw
        if not args.no_solves:
            out["time_to_1e8_junction"], flow = junction_time_to_1e8()
            if flow is not None:
                # the tracer carried by the converged flow, outlets held at zero
                # (the paper's case): GLS against Galerkin
                print("tracer on the junction", file=sys.stderr, flush=True)
                out["tracer_junction"] = tracer_junction_run(*flow, outlet_cases=("dirichlet",))
            out["junction_re500_pseudo_time"] = junction_re500_attempt(prob)
            out["mode_sweep"] = mode_sweep_200k()
            print("batched solves", file=sys.stderr, flush=True)
            out["batched"] = batched_run(64)
            print("learned warm start", file=sys.stderr, flush=True)
            out["learned"] = learned_run(512, 16, 64)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, m)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
