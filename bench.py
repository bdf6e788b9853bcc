"""Throughput of the batched functional-map solve (forward + backward) on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload headline|mixed|large|plain]

One step = one pass of the whole path over one batch of shape pairs already
resident in HBM: projection of both shapes of every pair (Eq. 1), mask, normal
products, per-row Cholesky solves (Eqs. 4-9), adjoint, projection backward.
The four library calls of a step are captured once in a HIP graph per input
set; K graph replays are timed with HIP events on the replay stream, rotating
over three copies of the inputs so that the reads are not served from the
256 MB last-level cache.

Prints ONE JSON line (metric, value = solves/s over the whole job, roofline of
the dominant kernel measured with HIP events, CPU oracle baseline, accuracy of
sampled pairs against the oracle).
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

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3       # MI355X dense float32 matrix
BF16_PEAK_TFLOPS = 2500.0      # MI355X dense bf16 matrix


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--warmup-seconds", type=float, default=1.5,
                    help="untimed replays for this much wall time before the counted warm-up")
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "plain", "mixed", "large", "ragged", "overlap", "gradfeat", "multires",
                             "vectorized"])
    ap.add_argument("--variant", default="A", choices=["A", "B"], help="gradient-feature variant (gradfeat)")
    ap.add_argument("--bwd", default=None, choices=["stored", "recompute"],
                    help="backward mode (default: recompute for the large workload, stored otherwise)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-graph", action="store_true", help="launch eagerly instead of replaying a HIP graph")
    ap.add_argument("--split", type=int, default=1,
                    help="sub-batches per step, staggered on their own streams (1: one sequence of calls)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-pair float32 leg")
    ap.add_argument("--oracle-one-pair", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cache-dir", default=None, help="keep generated workloads here (.npy) and reuse them")
    ap.add_argument("--pmc-summary", nargs="+", default=None, metavar="DIR",
                    help="only summarise rocprofv3 counter-collection output (mean per dispatch, per kernel)")
    ap.add_argument("--stats-summary", nargs="+", default=None, metavar="DIR",
                    help="only summarise rocprofv3 --stats kernel output")
    ap.add_argument("--trace-summary", nargs="+", default=None, metavar="DIR",
                    help="only summarise rocprofv3 --kernel-trace output per kernel and launch grid")
    ap.add_argument("--traffic-summary", nargs=4, default=None, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="only summarise FETCH_SIZE / WRITE_SIZE runs, calibrated by the --copy-probe runs")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many eager steps (for rocprofv3), no JSON")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run 3 plain device copies of 256 MiB (calibrates the HBM byte counters), no JSON")
    return ap.parse_args()


def make_workload(name: str, pairs=None):
    """The named workload; with --cache-dir, generated once and reloaded from .npy files afterwards (the
    profiler passes each start a fresh process)."""
    from paper_2604_10377_amd import synth
    kw = {} if pairs is None else {"pairs": pairs}
    cache = os.environ.get("FMAP_BENCH_CACHE")
    fields = ("phi", "mass", "feat", "evals", "lam", "dC", "phi_bf16", "feat_bf16")
    if cache and pairs is None:
        d = os.path.join(cache, name)
        if os.path.exists(os.path.join(d, "meta.json")):
            meta = json.load(open(os.path.join(d, "meta.json")))
            arr = {f: (np.load(os.path.join(d, f + ".npy")) if meta["has"][f] else None) for f in fields}
            return synth.PairBatch(meta["name"], meta["pairs"], meta["n"], meta["k"], meta["d"], meta["mask"],
                                   meta["gamma"], **arr)
    if name == "headline":
        b = synth.workload_headline(**kw)
    elif name == "plain":
        b = synth.workload_plain()
    elif name == "mixed":
        b = synth.workload_mixed(**kw)
    else:
        b = synth.workload_large(**kw)
    if cache and pairs is None:
        d = os.path.join(cache, name)
        os.makedirs(d, exist_ok=True)
        for f in fields:
            if getattr(b, f) is not None:
                np.save(os.path.join(d, f + ".npy"), getattr(b, f))
        json.dump({"name": b.name, "pairs": b.pairs, "n": b.n, "k": b.k, "d": b.d, "mask": b.mask, "gamma": b.gamma,
                   "has": {f: getattr(b, f) is not None for f in fields}}, open(os.path.join(d, "meta.json"), "w"))
    return b


# solve options per workload: the mixed-precision workload runs one float64-residual
# refinement step and forms A A^T in float64 when its condition estimate exceeds 1e6
SOLVE_OPTS = {"mixed": dict(refine_steps=1, cond_fp64_threshold=1e6)}


class Step:
    """Preallocated buffers and the four library calls of one forward + backward pass."""

    def __init__(self, F, dev, b, inputs, bwd="stored", refine_steps=0, cond_fp64_threshold=0.0):
        import torch
        self.F, self.b, self.bwd = F, b, bwd
        self.refine, self.cond_thr = refine_steps, cond_fp64_threshold
        P, n, k, d = b.pairs, b.n, b.k, b.d
        self.phi, self.mass, self.feat, self.ex, self.ey, self.lam, self.dC = inputs
        self.AB = torch.empty((2 * P, k, d), dtype=torch.float32, device=dev)
        self.C = torch.empty((P, k, k), dtype=torch.float32, device=dev)
        self.info = torch.empty((P, k), dtype=torch.int32, device=dev)
        self.fac = (torch.empty((P, F.fmap_factor_floats(k, k)), dtype=torch.float32, device=dev)
                    if bwd == "stored" or refine_steps > 0 else None)
        self.dAB = torch.empty_like(self.AB)
        self.dF = torch.empty((2 * P, n, d), dtype=torch.float32, device=dev)
        dt = F.FMAP_BF16 if self.phi.dtype == torch.bfloat16 else F.FMAP_F32
        self.wsp = torch.empty(max(F.fmap_project_workspace_bytes(2 * P, n, k, d, dt), 256), dtype=torch.uint8,
                               device=dev)
        self.wss = torch.empty(F.fmap_solve_workspace_bytes(P, k, k, d), dtype=torch.uint8, device=dev)

    def project(self):
        self.F.fmap_project(self.phi, self.mass, self.feat, A=self.AB, workspace=self.wsp)

    def solve(self):
        P, b = self.b.pairs, self.b
        self.F.fmap_solve(self.AB[:P], self.AB[P:], self.ex, self.ey, self.lam, b.mask, b.gamma, C=self.C,
                          factors=self.fac, info=self.info, workspace=self.wss, store_factors=self.fac is not None,
                          refine_steps=self.refine, cond_fp64_threshold=self.cond_thr)

    def solve_backward(self):
        P, b = self.b.pairs, self.b
        self.F.fmap_solve_backward(self.dC, self.AB[:P], self.AB[P:], self.C, self.ex, self.ey, self.lam, b.mask,
                                   b.gamma, self.fac if self.bwd == "stored" else None, dA=self.dAB[:P],
                                   dB=self.dAB[P:], workspace=self.wss)

    def project_backward(self):
        self.F.fmap_project_backward(self.phi, self.mass, self.dAB, dF=self.dF)

    def run(self):
        self.project()
        self.solve()
        if self.dC is not None:
            self.solve_backward()
            self.project_backward()


def phase_costs(b, bf16: bool):
    """Algorithmic flops and HBM bytes of each phase for the whole batch (see DESIGN)."""
    P, n, k, d = b.pairs, b.n, b.k, b.d
    S = 2 * P
    eb = 2 if bf16 else 4
    proj_flops = 2.0 * n * k * d * S
    proj_bytes = S * (n * k * eb + n * d * eb + n * 4 + k * d * 4)
    tri = k * (k + 1) // 2
    solve_flops = P * (3.0 * k * k * d + k ** 4 / 3.0 + 2.0 * k ** 3)
    solve_bytes = P * (2 * k * d * 4 + 2 * k * 4 + 4 + k * k * 4 + k * tri * 4 + k * 4)
    adj_flops = P * (4.0 * k ** 3 + 6.0 * k * k * d)
    adj_bytes = P * (k * k * 4 * 2 + 2 * k * d * 4 + k * tri * 4 + 2 * k * d * 4)
    pbwd_flops = proj_flops
    pbwd_bytes = S * (n * k * eb + n * 4 + k * d * 4 + n * d * 4)
    return {"project": (proj_flops, proj_bytes), "solve": (solve_flops, solve_bytes),
            "solve_backward": (adj_flops, adj_bytes), "project_backward": (pbwd_flops, pbwd_bytes)}


def matrix_peak(phase: str, b, bf16: bool):
    """(TFLOP/s of useful products, note) for the matrix cores the library dispatches for this phase.

    The bf16 paths run the bf16 matrix cores (2500 TFLOP/s dense) with more than one bf16 product per
    useful product: basis x mass (forward) or dA (backward) split in two, or, for float32 operands,
    both operands split in three with six products kept.  Shapes outside those paths use the float32
    matrix cores (157.3 TFLOP/s)."""
    n, k, d = b.n, b.k, b.d
    if phase == "project":
        if bf16 and k % 8 == 0 and 8 <= k <= 256 and d % 8 == 0 and n % 4 == 0 and n >= 128:
            return BF16_PEAK_TFLOPS / 2, "bf16 matrix cores, 2 bf16 products per product"
        kok = (k % 2 == 0 and 4 <= k <= 64) or (k % 4 == 0 and 64 < k <= 319)
        if not bf16 and kok and d % 4 == 0 and n % 4 == 0 and n >= 128:
            return BF16_PEAK_TFLOPS / 6, "bf16 matrix cores, float32 emulated with 6 bf16 products"
        return FP32_PEAK_TFLOPS, "float32 matrix cores"
    if phase == "project_backward":
        if bf16 and k % 8 == 0 and 8 <= k <= 256:
            return BF16_PEAK_TFLOPS / 2, "bf16 matrix cores, 2 bf16 products per product"
        if not bf16 and k % 2 == 0 and 2 <= k <= 319:
            return BF16_PEAK_TFLOPS / 6, "bf16 matrix cores, float32 emulated with 6 bf16 products"
        return FP32_PEAK_TFLOPS, "float32 matrix cores"
    return FP32_PEAK_TFLOPS, "float32"


def roofline_entry(flops, nbytes, seconds, mfma_peak_tflops):
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    t_mfma = flops / (mfma_peak_tflops * 1e12)
    if t_mfma >= t_hbm:
        ach = flops / seconds / 1e12
        return {"bound": "mfma", "achieved": round(ach, 2), "peak": mfma_peak_tflops, "unit": "TFLOP/s",
                "frac": round(ach / mfma_peak_tflops, 4)}
    ach = nbytes / seconds / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4)}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "headline_hbm_traffic.txt")
KERNEL_OF_PHASE = {"project": "fmap::proj_fwd_x3r_kernel<false>",
                   "project_backward": "fmap::proj_bwd_mc_kernel<float, 3, 3, 2>"}


def measured_traffic(phase: str, workload: str, pairs_per_launch: int):
    """HBM bytes per launch of the phase's main kernel from the committed byte-counter summary.

    None unless the summary covers this workload at this launch size (its "shapes per launch" line) and
    the kernel source still has the hash the counters were taken with (a changed kernel voids them)."""
    import hashlib
    if workload != "headline" or phase not in KERNEL_OF_PHASE or not os.path.exists(TRAFFIC_FILE):
        return None
    lines = open(TRAFFIC_FILE).read().splitlines()
    per = [ln for ln in lines if ln.startswith("shapes per launch: ")]
    if not per or int(per[0].split(":")[1]) != 2 * pairs_per_launch:
        return None
    src = [ln for ln in lines if ln.startswith("source: ")]
    if not src:
        return None
    rel, _, want = src[0][len("source: "):].split()[:3]
    have = hashlib.sha256(open(os.path.join(ROOT, rel), "rb").read()).hexdigest()[:16]
    if have != want:
        return None
    name = KERNEL_OF_PHASE[phase]
    for ln in lines:
        if ln.startswith(name + " ") or ln.startswith("void " + name + " "):
            read_mb, write_mb = (float(x) for x in ln.split()[-2:])
            return {"bytes": round((read_mb + write_mb) * 1e6), "read_MB": read_mb, "write_MB": write_mb,
                    "kernel": name, "source_sha256": want}
    return None


def warm_up(replay, args):
    """Untimed replays for --warmup-seconds of wall time (the GPU's clocks settle under sustained load;
    a short burst right after set-up runs slower), then the W counted warm-up steps."""
    import torch
    t0, i = time.perf_counter(), 0
    while time.perf_counter() - t0 < args.warmup_seconds:
        for _ in range(10):
            replay(i)
            i += 1
        torch.cuda.synchronize()
    for j in range(args.warmup):
        replay(i + j)
    torch.cuda.synchronize()


def timed_steps(replay, K, stream):
    """K steps between events on the replay stream, one event after each step.

    Returns (mean ms per step over the whole timed region, per-step statistics)."""
    import torch
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    for i in range(K):
        replay(i)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(K)])
    ms = evs[0].elapsed_time(evs[K]) / K
    stats = {"median": round(float(np.median(per)), 5), "p10": round(float(np.percentile(per, 10)), 5),
             "p90": round(float(np.percentile(per, 90)), 5), "mean": round(ms, 5)}
    return ms, stats


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def single_core_pair(workload: str):
    """Seconds the oracle takes for pair 0 of the workload (forward + backward, full n) on one thread, in a
    child process started with OMP_NUM_THREADS=1 (it never touches the GPU)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-one-pair", "--workload", workload],
                       capture_output=True, text=True, env=env, timeout=600)
    if r.returncode != 0:
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def oracle_one_pair(workload: str):
    import oracle
    b = make_workload(workload, pairs=1)
    args = (b.phi_consumed(), b.mass, b.feat_consumed(), b.evals, b.lam, b.mask, b.gamma, b.dC)
    t0 = time.perf_counter()
    oracle.pipeline_batch(*args)
    print(json.dumps({"seconds": round(time.perf_counter() - t0, 3), "threads": oracle.num_threads()}), flush=True)


def cpu_baseline(b, seconds: float, workload: str):
    """The oracle, as it stands, on a bounded sample of the same workload (whole pairs, full n), on every
    host core this process may use; plus one pair on one core."""
    import oracle
    P = b.pairs
    npairs = max(1, min(P, 4))
    sel = list(range(npairs))
    idx = sel + [P + p for p in sel]
    args = (b.phi_consumed()[idx], b.mass[idx], b.feat_consumed()[idx], b.evals[idx], b.lam[sel], b.mask, b.gamma,
            b.dC[sel])
    done, t0 = 0, time.perf_counter()
    while True:
        oracle.pipeline_batch(*args)
        done += npairs
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    one = single_core_pair(workload)
    return {"value": round(done / el, 3), "unit": "solves/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{done} solves ({npairs}-pair batches of the {b.name} workload, full n) in {el:.1f} s, fp64",
            "cpu_model": cpu_model(), "affinity_cores": len(os.sched_getaffinity(0)),
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS"),
            "one_pair_one_core_s": None if one is None else one["seconds"]}


def accuracy(b, split, pairs=(0, 1)):
    """Relative Frobenius error of C and dF of sampled pairs against the oracle (pairs located in their
    sub-batch of the split step)."""
    P = b.pairs
    out = {}
    for p in pairs:
        st, q = split.locate(p)
        out[p] = (st.C[q].cpu().numpy(), None if b.dC is None else
                  (st.dF[q].cpu().numpy(), st.dF[st.b.pairs + q].cpu().numpy()))
    return _errors(b, out)


def accuracy_plain(b, psteps, pairs):
    out = {}
    for p in pairs:
        st = psteps[p][0]
        out[p] = (st.C[0].cpu().numpy(), None if b.dC is None else (st.dF[0].cpu().numpy(),
                                                                   st.dF[1].cpu().numpy()))
    return _errors(b, out)


def _errors(b, got):
    import oracle
    P = b.pairs
    phi, feat = b.phi_consumed(), b.feat_consumed()
    worst = {"C": 0.0, "dF": 0.0}
    rel = lambda x, r: float(np.linalg.norm(x - r) / np.linalg.norm(r))
    for p, (C, dF) in got.items():
        A, B, D, Cr, _ = oracle.forward_pair(phi[p], b.mass[p], feat[p], phi[P + p], b.mass[P + p], feat[P + p],
                                             b.evals[p], b.evals[P + p], float(b.lam[p]), b.mask, b.gamma)
        worst["C"] = max(worst["C"], rel(C, Cr))
        if dF is None:
            continue  # forward-only workload
        dA, dB, _ = oracle.solve_backward(A, B, Cr, D, float(b.lam[p]), b.dC[p])
        worst["dF"] = max(worst["dF"], rel(dF[0], oracle.project_backward(phi[p], b.mass[p], dA)),
                          rel(dF[1], oracle.project_backward(phi[P + p], b.mass[P + p], dB)))
    if b.dC is None:
        worst.pop("dF")
    return {k: float(f"{v:.3e}") for k, v in worst.items()} | {"pairs": sorted(got)}


def ragged_costs(pairs, d):
    """Algorithmic (flops, bytes, matrix-core seconds) of one forward and one backward pass over an uneven
    batch, summed per pair; each flop is priced at the peak of the cores the plan runs it on."""
    from types import SimpleNamespace
    tot = {"fwd": [0.0, 0.0, 0.0], "bwd": [0.0, 0.0, 0.0]}

    def add(key, flops, nbytes, peak):
        tot[key][0] += flops
        tot[key][1] += nbytes
        tot[key][2] += flops / (peak * 1e12)

    for p in pairs:
        for n in (p.n_x, p.n_y):
            sb = SimpleNamespace(pairs=1, n=n, k=p.k, d=d)
            c = phase_costs(sb, False)
            # phase_costs counts a pair (two shapes of n vertices): halve the projection terms per shape
            # the plan runs whole 32-vertex stages of any n on the emulated kernel: price by k and d only
            add("fwd", c["project"][0] / 2, c["project"][1] / 2,
                matrix_peak("project", SimpleNamespace(pairs=1, n=128, k=p.k, d=d), False)[0])
            add("bwd", c["project_backward"][0] / 2, c["project_backward"][1] / 2,
                matrix_peak("project_backward", sb, False)[0])
        c = phase_costs(SimpleNamespace(pairs=1, n=0, k=p.k, d=d), False)
        add("fwd", c["solve"][0], c["solve"][1], FP32_PEAK_TFLOPS)
        add("bwd", c["solve_backward"][0], c["solve_backward"][1], FP32_PEAK_TFLOPS)
    return tot


def bench_ragged(args, F, dev):
    """Uneven batch through one plan: captured forward + backward graphs, replayed K times."""
    import tempfile

    import torch
    from paper_2604_10377_amd import synth
    pairs = synth.workload_ragged()
    d = 256
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    dp = [dict(phi_x=t(p.phi_x), phi_y=t(p.phi_y), mass_x=t(p.mass_x), mass_y=t(p.mass_y), feat_x=t(p.feat_x),
               feat_y=t(p.feat_y), evals_x=t(p.evals_x), evals_y=t(p.evals_y), lam=t(np.asarray([p.lam])))
          for p in pairs]
    bwd = args.bwd or "stored"
    cache = os.path.join(tempfile.gettempdir(), "fmap_tune_cache.txt")
    t0 = time.perf_counter()
    plan = F.FmapPlan(dp, synth.MASK_LAPLACIAN, 0.5, backward=True, recompute=(bwd == "recompute"),
                      tune_cache=cache)
    create_s = time.perf_counter() - t0
    for i, p in enumerate(pairs):
        plan.dC[i].copy_(torch.from_numpy(p.dC))
    stream = torch.cuda.current_stream(dev)

    def step():
        plan.forward()
        plan.backward()

    if args.profile_steps:
        for _ in range(args.profile_steps):
            step()
        torch.cuda.synchronize()
        print(f"profiled {args.profile_steps} plan steps of the ragged workload", flush=True)
        return
    warm_up(lambda i: step(), args)
    ms, step_stats = timed_steps(lambda i: step(), args.steps, stream)
    # forward and backward graphs timed separately
    pass_ms = {}
    for name, fn in (("fwd", plan.forward), ("bwd", plan.backward)):
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(20):
            fn()
        z.record(stream)
        torch.cuda.synchronize()
        pass_ms[name] = a.elapsed_time(z) / 20
    costs = ragged_costs(pairs, d)
    dom = max(pass_ms, key=pass_ms.get)
    fl, by, tm = costs[dom]
    roof = roofline_entry(fl, by, pass_ms[dom] * 1e-3, fl / tm / 1e12)  # effective peak of the pass's mix
    roof["kernel"] = f"plan {dom} pass (graph: projection items on the emulated float32 kernels + grouped solves)"
    roof["traffic"] = None
    roof["pass_us"] = {k: round(v * 1e3, 2) for k, v in pass_ms.items()}
    t_roof = sum(max(t, b_ / (HBM_PEAK_GBS * 1e9)) for _, b_, t in costs.values())
    roof["step_roofline_us"] = round(t_roof * 1e6, 2)
    roof["step_frac"] = round(t_roof * 1e3 / ms, 4)
    # accuracy of sampled pairs
    import oracle
    worst = {"C": 0.0, "dF": 0.0}
    rel = lambda x, r: float(np.linalg.norm(x - r) / np.linalg.norm(r))
    for i in (0, len(pairs) - 1):
        p = pairs[i]
        A, B, D, Cr, _ = oracle.forward_pair(p.phi_x, p.mass_x, p.feat_x, p.phi_y, p.mass_y, p.feat_y, p.evals_x,
                                             p.evals_y, p.lam, synth.MASK_LAPLACIAN, 0.5)
        dA, dB, _ = oracle.solve_backward(A, B, Cr, D, p.lam, p.dC)
        worst["C"] = max(worst["C"], rel(plan.C[i].cpu().numpy(), Cr))
        worst["dF"] = max(worst["dF"], rel(plan.dF_x[i].cpu().numpy(), oracle.project_backward(p.phi_x, p.mass_x, dA)),
                          rel(plan.dF_y[i].cpu().numpy(), oracle.project_backward(p.phi_y, p.mass_y, dB)))
    ks = sorted({p.k for p in pairs})
    out = {
        "metric": "functional map solves/sec (fwd+bwd), uneven batch",
        "value": round(len(pairs) / (ms * 1e-3), 1),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "step_ms": step_stats,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ragged-k30..120-d256", "pairs": len(pairs), "n_range": [min(min(p.n_x, p.n_y)
                   for p in pairs), max(max(p.n_x, p.n_y) for p in pairs)], "k_values": ks,
                   "k_counts": {str(k): sum(p.k == k for p in pairs) for k in ks}, "d": d, "mask": "laplacian",
                   "backward": bwd, "graph": True},
        "tuning": plan.tuning() | {"create_s": round(create_s, 2)},
        "roofline": roof,
        "cpu_baseline": None,
        "accuracy_vs_oracle": {k: float(f"{v:.3e}") for k, v in worst.items()} | {"pairs": [0, len(pairs) - 1]},
    }
    print(json.dumps(out), flush=True)
    plan.close()


class SplitStep:
    """One step as S sub-batches of consecutive pairs on S streams (default priority), staggered: sub-batch
    j starts its projection when sub-batch j - 1's projection is done, so the latency-bound solve and
    adjoint of one sub-batch run beside the HBM-bound projections of its neighbours.  S = 1 is the plain
    sequence of the four library calls.  Captured once as a graph, the streams become graph branches."""

    def __init__(self, steps, side_streams):
        self.steps, self.side = steps, side_streams

    def run(self):
        # the sub-batches fork from the stream current at the call (under graph capture: the capture
        # stream) and join it again at the end
        import torch
        main = torch.cuda.current_stream()
        streams = [main] + list(self.side)
        prev = None
        for j, (st, s) in enumerate(zip(self.steps, streams)):
            if j > 0:
                s.wait_event(prev)
            with torch.cuda.stream(s):
                st.project()
                prev = torch.cuda.Event()
                prev.record(s)
                st.solve()
                if st.dC is not None:
                    st.solve_backward()
                    st.project_backward()
        for s in streams[1:]:
            main.wait_stream(s)

    def locate(self, p):
        """(sub-batch step, index within it) of pair p."""
        for st in self.steps:
            if p < st.b.pairs:
                return st, p
            p -= st.b.pairs
        raise IndexError(p)


def split_pairs(P: int, S: int):
    """S consecutive ranges of pairs, sizes differing by at most one."""
    S = max(1, min(S, P))
    edges = [round(j * P / S) for j in range(S + 1)]
    return [list(range(edges[j], edges[j + 1])) for j in range(S)]


def sub_batch(b, npairs):
    from types import SimpleNamespace
    return SimpleNamespace(pairs=npairs, n=b.n, k=b.k, d=b.d, mask=b.mask, gamma=b.gamma, name=b.name)


def plain_leg(args, F, b, dev, inputs, opts):
    """The plain float32 GPU path: per-pair library calls (two projections, solve, adjoint, two projection
    backwards), launched eagerly, no graph, factors stored.  Timed over whole steps like the batched form;
    returns (solves/s, ms per step, errors of sampled pairs against the oracle)."""
    import torch
    phi, mass, feat, ex, ey, lam, dC = inputs
    P, k, d = b.pairs, b.k, b.d
    one = sub_batch(b, 1)
    steps = []
    for p in range(P):
        sl = lambda t, i: t[i:i + 1]
        stx = Step(F, dev, one, (sl(phi, p), sl(mass, p), sl(feat, p), sl(ex, p), sl(ey, p), sl(lam, p),
                                 None if dC is None else sl(dC, p)), "stored", **opts)
        sty = (sl(phi, P + p), sl(mass, P + p), sl(feat, P + p))
        steps.append((stx, sty))
    dev_AB = [torch.empty((2, k, d), dtype=torch.float32, device=dev) for _ in range(P)]

    def run():
        for p, (st, (py, my, fy)) in enumerate(steps):
            AB = dev_AB[p]
            F.fmap_project(st.phi, st.mass, st.feat, A=AB[:1], workspace=st.wsp)
            F.fmap_project(py, my, fy, A=AB[1:], workspace=st.wsp)
            F.fmap_solve(AB[:1], AB[1:], st.ex, st.ey, st.lam, b.mask, b.gamma, C=st.C, factors=st.fac,
                         info=st.info, workspace=st.wss, store_factors=True, refine_steps=st.refine,
                         cond_fp64_threshold=st.cond_thr)
            if st.dC is not None:
                F.fmap_solve_backward(st.dC, AB[:1], AB[1:], st.C, st.ex, st.ey, st.lam, b.mask, b.gamma, st.fac,
                                      dA=st.dAB[:1], dB=st.dAB[1:], workspace=st.wss)
                F.fmap_project_backward(st.phi, st.mass, st.dAB[:1], dF=st.dF[:1])
                F.fmap_project_backward(py, my, st.dAB[1:], dF=st.dF[1:])

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.5:
        run()
        torch.cuda.synchronize()
    K = max(3, min(args.steps, 20))
    ms, stats = timed_steps(lambda i: run(), K, torch.cuda.current_stream(dev))
    return P / (ms * 1e-3), ms, stats, steps


def timed_calls(fn, args, stream):
    """Warm-up (time-based, then W calls) and K calls between per-call events: (mean ms, stats)."""
    warm_up(lambda i: fn(), args)
    return timed_steps(lambda i: fn(), args.steps, stream)


def bench_overlap(args, F, dev):
    """Overlap metrics of an evaluation batch (1024 shapes of 2000-20000 vertices): one call per step."""
    import torch
    from oracle import overlap as ov
    from paper_2604_10377_amd import synth
    b = synth.workload_overlap()
    S, total = b.offsets.shape[0] - 1, int(b.offsets[-1])
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    sc, tr, off = t(b.scores), t(b.truth), t(b.offsets)
    counts = torch.empty((S, 4), dtype=torch.int64, device=dev)
    mets = torch.empty((S, 7), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    call = lambda: F.fmap_overlap_metrics(sc, tr, off, 0.5, counts=counts, metrics=mets)
    if args.profile_steps:
        for _ in range(args.profile_steps):
            call()
        torch.cuda.synchronize()
        print(f"profiled {args.profile_steps} overlap-metric calls", flush=True)
        return
    ms, stats = timed_calls(call, args, stream)
    nbytes = total * 5 + 8 * (S + 1) + S * (4 * 8 + 7 * 4)
    roof = roofline_entry(0.0, nbytes, ms * 1e-3, FP32_PEAK_TFLOPS)
    roof["kernel"] = "fmap_overlap_metrics (clear, count, metrics kernels; the count pass carries the bytes)"
    roof["traffic"] = None
    counts.zero_()
    call()
    torch.cuda.synchronize()
    c, m = counts.cpu().numpy(), mets.cpu().numpy()
    sel = list(range(0, S, max(1, S // 16)))
    exact = True
    for s_ in sel:
        a, z = int(b.offsets[s_]), int(b.offsets[s_ + 1])
        rc = ov.confusion_counts(b.scores[a:z], b.truth[a:z], 0.5)
        exact &= tuple(c[s_]) == rc and np.array_equal(m[s_], ov.metrics_from_counts(*rc).astype(np.float32))
    cpu = None
    if not args.no_cpu_baseline:
        t0, done = time.perf_counter(), 0
        while time.perf_counter() - t0 < min(args.cpu_seconds, 5.0):
            ov.overlap_batch(b.scores[:b.offsets[64]], b.truth[:b.offsets[64]], b.offsets[:65], 0.5)
            done += 64
        el = time.perf_counter() - t0
        cpu = {"value": round(done / el, 1), "unit": "shapes/s", "cores": 1, "kind": "oracle",
               "sample": f"{done} shapes (the first 64 of the batch, repeated) in {el:.1f} s, numpy float64",
               "cpu_model": cpu_model()}
    out = {"metric": "overlap-metric evaluations/sec (confusion counts + 7 metrics per shape)",
           "value": round(S / (ms * 1e-3), 1), "unit": "shapes/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 5), "step_ms": stats, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32-scores/u8-labels/i64-counts", "data": "synthetic",
           "config": {"workload": "overlap-1024", "shapes": S, "vertices": total, "threshold": 0.5},
           "roofline": roof, "cpu_baseline": cpu,
           "accuracy_vs_oracle": {"bit_exact": bool(exact), "shapes_checked": len(sel)}}
    print(json.dumps(out), flush=True)


def bench_gradfeat(args, F, dev):
    """Spatial-gradient features of the headline batch's vertices (160000 x 128 channels): one call per step."""
    import torch
    from oracle import gradfeat as gf
    from paper_2604_10377_amd import synth
    z, Ar, Ai = synth.workload_gradfeat()
    V, D = z.shape[0], z.shape[1]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    # three input copies, rotated, so that the z reads are not served from the last-level cache
    zs = [t(z)] + [t(z).clone() for _ in range(2)]
    tAr, tAi = t(Ar), t(Ai)
    g = torch.empty((V, D), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    k = [0]

    def call():
        F.fmap_gradient_features(zs[k[0] % 3], tAr, tAi, args.variant, g=g)
        k[0] += 1

    if args.profile_steps:
        for _ in range(args.profile_steps):
            call()
        torch.cuda.synchronize()
        print(f"profiled {args.profile_steps} gradient-feature calls", flush=True)
        return
    ms, stats = timed_calls(call, args, stream)
    flops = 8.0 * D * D * V + 3.0 * D * V
    nbytes = V * D * 12 + 2 * D * D * 4
    roof = roofline_entry(flops, nbytes, ms * 1e-3, FP32_PEAK_TFLOPS)
    roof["kernel"] = f"gradfeat_mfma_kernel<{D}> (float32 matrix cores)"
    roof["traffic"] = None
    F.fmap_gradient_features(zs[0], tAr, tAi, args.variant, g=g)
    torch.cuda.synchronize()
    rows = np.random.default_rng(0).choice(V, 2000, replace=False)
    ref = gf.gradient_features(z[rows], Ar, Ai, args.variant)
    got = g.cpu().numpy()[rows]
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    cpu = None
    if not args.no_cpu_baseline:
        t0, done = time.perf_counter(), 0
        while time.perf_counter() - t0 < min(args.cpu_seconds, 5.0):
            gf.gradient_features(z[:20000], Ar, Ai, args.variant)
            done += 20000
        el = time.perf_counter() - t0
        cpu = {"value": round(done / el, 1), "unit": "vertices/s", "cores": int(os.environ.get("OMP_NUM_THREADS", 0))
               or len(os.sched_getaffinity(0)), "kind": "oracle",
               "sample": f"{done} vertices (20000-vertex slices) in {el:.1f} s, numpy float64 (BLAS threads)",
               "cpu_model": cpu_model()}
    out = {"metric": f"spatial-gradient feature vertices/sec (variant {args.variant}, D={D})",
           "value": round(V / (ms * 1e-3), 1), "unit": "vertices/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 5), "step_ms": stats, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"gradfeat-v{V}-d{D}", "vertices": V, "channels": D, "variant": args.variant},
           "roofline": roof, "cpu_baseline": cpu,
           "accuracy_vs_oracle": {"g": float(f"{err:.3e}"), "rows_checked": len(rows)}}
    print(json.dumps(out), flush=True)


def bench_vectorized(args, F, dev):
    """The vectorized solve with general commutativity operators: 256 pairs, kx = ky = 16 (normal equations of
    order n = 256 per pair), d = 256, lambda = 0.1, non-symmetric operators; one library call per step."""
    import torch
    from oracle import vectorized as vz
    from paper_2604_10377_amd import synth
    A, B, D1, D2, lam = synth.workload_vectorized()
    P, kx, d = A.shape
    ky = B.shape[1]
    n = kx * ky
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    tA, tB, tD1, tD2, tl = t(A), t(B), t(D1), t(D2), t(lam)
    ws = torch.empty(max(F.fmap_solve_vectorized_workspace_bytes(P, kx, ky, d), 256), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    out = [None]

    def call():
        out[0] = F.fmap_solve_vectorized(tA, tB, tD1, tD2, tl, workspace=ws)

    if args.profile_steps:
        for _ in range(args.profile_steps):
            call()
        torch.cuda.synchronize()
        print(f"profiled {args.profile_steps} vectorized-solve calls", flush=True)
        return
    ms, stats = timed_calls(call, args, stream)
    # algorithmic work per pair: Cholesky n^3/3 and the two substitutions 2 n^2 (multiply-adds x 2), the
    # products A A^T and B A^T 2 (kx^2 + ky kx) d; bytes: A, B, the operators, H written and read, C
    flops = P * (2.0 * (n ** 3 / 3.0 + 2.0 * n * n) + 2.0 * (kx * kx + ky * kx) * d)
    nbytes = P * 4.0 * ((kx + ky) * d + kx * kx + ky * ky + 2.0 * n * n + 2.0 * n)
    roof = roofline_entry(flops, nbytes, ms * 1e-3, FP32_PEAK_TFLOPS)
    roof["kernel"] = "whole call: normal products, vec_form_kernel, rowsolve_ll_kernel<10> (one system per pair)"
    roof["traffic"] = None
    call()
    torch.cuda.synchronize()
    C, info = out[0][0].cpu().numpy(), out[0][1].cpu().numpy()
    assert (info == 0).all(), info
    errs = [float(np.linalg.norm(C[p] - vz.solve(A[p], B[p], D1[p], D2[p], float(lam[p])))
                  / np.linalg.norm(vz.solve(A[p], B[p], D1[p], D2[p], float(lam[p])))) for p in (0, P - 1)]
    cpu = None
    if not args.no_cpu_baseline:
        t0, done = time.perf_counter(), 0
        while time.perf_counter() - t0 < min(args.cpu_seconds, 5.0):
            vz.solve(A[done % P], B[done % P], D1[done % P], D2[done % P], float(lam[done % P]))
            done += 1
        el = time.perf_counter() - t0
        cpu = {"value": round(done / el, 2), "unit": "solves/s", "cores": int(os.environ.get("OMP_NUM_THREADS", 0))
               or len(os.sched_getaffinity(0)), "kind": "oracle",
               "sample": f"{done} pairs of the same batch in {el:.1f} s, numpy float64 (Kronecker system + LU)",
               "cpu_model": cpu_model()}
    res = {"metric": f"vectorized-operator solves/sec (kx=ky={kx}, n={n}, d={d}, batch {P})",
           "value": round(P / (ms * 1e-3), 1), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 5), "step_ms": stats, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"vectorized-k{kx}-d{d}", "pairs": P, "kx": kx, "ky": ky, "d": d,
                      "lambda": float(lam[0]), "operators": "Q diag(mu) Q^-1, Q = I + 0.1 N"},
           "roofline": roof, "cpu_baseline": cpu,
           "accuracy_vs_oracle": {"C": float(f"{max(errs):.3e}"), "pairs": [0, P - 1]}}
    print(json.dumps(res), flush=True)


def bench_multires(args, F, dev):
    """One projection at k = 120 and maps at resolutions 30, 50, 80 and 120 (32 pairs, n = 5000, d = 256,
    Laplacian mask): the two library calls captured as one graph per input set, three sets rotated."""
    import torch
    import oracle
    from paper_2604_10377_amd import synth
    b = synth.make_batch("multires-k120-d256", 14, 32, 5000, 120, 256, mask=synth.MASK_LAPLACIAN, with_grad=False)
    P, n, k, d = b.pairs, b.n, b.k, b.d
    res = [(30, 30), (50, 50), (80, 80), (120, 120)]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    sets = [(t(b.phi), t(b.mass), t(b.feat)) for _ in range(3)]
    ex, ey, lam = t(b.evals_x), t(b.evals_y), t(b.lam)
    AB = [torch.empty((2 * P, k, d), dtype=torch.float32, device=dev) for _ in range(3)]
    wsp = torch.empty(max(F.fmap_project_workspace_bytes(2 * P, n, k, d), 256), dtype=torch.uint8, device=dev)
    outs = [None] * 3

    def run(i):
        phi, mass, feat = sets[i % 3]
        F.fmap_project(phi, mass, feat, A=AB[i % 3], workspace=wsp)
        outs[i % 3] = F.fmap_solve_resolutions(AB[i % 3][:P], AB[i % 3][P:], ex, ey, lam, b.mask, b.gamma, res)

    for i in range(3):
        run(i)
    torch.cuda.synchronize()
    if args.profile_steps:
        for i in range(args.profile_steps):
            run(i)
        torch.cuda.synchronize()
        print(f"profiled {args.profile_steps} eager multi-resolution steps", flush=True)
        return
    graphs = []
    for i in range(3):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            run(i)
        graphs.append(g)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    replay = lambda i: graphs[i % 3].replay()
    warm_up(replay, args)
    ms, stats = timed_steps(replay, args.steps, stream)
    # phases alone (eager): projection, then the four solves
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    K = max(3, min(args.steps, 50))
    tp = ts = 0.0
    for i in range(K):
        phi, mass, feat = sets[i % 3]
        e[0].record(stream)
        F.fmap_project(phi, mass, feat, A=AB[0], workspace=wsp)
        e[1].record(stream)
        F.fmap_solve_resolutions(AB[0][:P], AB[0][P:], ex, ey, lam, b.mask, b.gamma, res)
        e[2].record(stream)
        torch.cuda.synchronize()
        tp += e[0].elapsed_time(e[1]) / K
        ts += e[1].elapsed_time(e[2]) / K
    sb = SimpleNamespace_(pairs=P, n=n, k=k, d=d)
    flops, nbytes = phase_costs(sb, False)["project"]
    roof = roofline_entry(flops, nbytes, tp * 1e-3, matrix_peak("project", sb, False)[0])
    roof["kernel"] = "fmap_project at k = 120 (float32 emulated on the bf16 matrix cores)"
    roof["traffic"] = None
    roof["phase_us"] = {"project": round(tp * 1e3, 2), "solve_resolutions": round(ts * 1e3, 2)}
    # accuracy of pairs 0 and P-1 at every resolution, from one replay into NaN-filled outputs
    for C, info in outs[0]:
        C.fill_(float("nan"))
    replay(0)
    torch.cuda.synchronize()
    worst = 0.0
    rel = lambda x, r: float(np.linalg.norm(x - r) / np.linalg.norm(r))
    for p in (0, P - 1):
        A = oracle.project(b.phi[p], b.mass[p], b.feat[p])
        B = oracle.project(b.phi[P + p], b.mass[P + p], b.feat[P + p])
        refs = oracle.solve_resolutions(A, B, b.evals_x[p], b.evals_y[p], float(b.lam[p]), b.mask, b.gamma,
                                        [r[0] for r in res], [r[1] for r in res])
        for (C, _), (Cr, _) in zip(outs[0], refs):
            worst = max(worst, rel(C[p].cpu().numpy(), Cr))
    out = {"metric": "multi-resolution functional map sets/sec (projection at k=120 + maps at k=30,50,80,120)",
           "value": round(P / (ms * 1e-3), 1), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 5), "step_ms": stats, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": b.name, "pairs": P, "n": n, "k_max": k, "d": d, "resolutions": res,
                      "mask": "laplacian", "graph": True},
           "roofline": roof, "cpu_baseline": None,
           "accuracy_vs_oracle": {"C": float(f"{worst:.3e}"), "pairs": [0, P - 1], "resolutions": len(res)}}
    print(json.dumps(out), flush=True)


def SimpleNamespace_(**kw):
    from types import SimpleNamespace
    return SimpleNamespace(**kw)


def short_kernel_name(name: str) -> str:
    """A kernel's name without its argument list (template arguments kept)."""
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0 and i > 0:
            return name[:i].strip()
    return name.strip()


def csv_files(paths, suffix):
    import glob
    out = []
    for pth in paths:
        out += sorted(glob.glob(os.path.join(pth, "**", "*" + suffix), recursive=True)) if os.path.isdir(pth) \
            else [pth]
    return out


def counter_means(paths):
    """{(kernel, counter): mean value per dispatch} from rocprofv3 counter-collection CSVs."""
    import csv
    acc = {}
    for f in csv_files(paths, "counter_collection.csv"):
        for row in csv.DictReader(open(f)):
            kn = short_kernel_name(row["Kernel_Name"])
            per = acc.setdefault((kn, row["Counter_Name"]), {})
            d = row["Dispatch_Id"]
            per[d] = per.get(d, 0.0) + float(row["Counter_Value"])  # summed over the dimensions of one dispatch
            if "Start_Timestamp" in row and "End_Timestamp" in row:
                acc.setdefault((kn, "duration_us"), {})[d] = \
                    (float(row["End_Timestamp"]) - float(row["Start_Timestamp"])) / 1e3
    return {k: (sum(v.values()) / len(v), len(v)) for k, v in acc.items()}


def pmc_summary(paths):
    """Mean value per dispatch of every counter, per kernel; with the matrix-core and LDS counters, the
    derived utilisation figures."""
    m = counter_means(paths)
    kernels = sorted({k for k, _ in m}, key=lambda k: -max(v[0] for (kk, _), v in m.items() if kk == k))
    counters = sorted({c for _, c in m})
    print("kernel".ljust(56) + "disp" + "".join(c.rjust(30) for c in counters))
    for kn in kernels:
        nd = max(m[(kn, c)][1] for c in counters if (kn, c) in m)
        vals = [f"{m[(kn, c)][0]:.4g}" if (kn, c) in m else "-" for c in counters]
        print(kn[:55].ljust(56) + str(nd).rjust(4) + "".join(v.rjust(30) for v in vals))
    if any(c == "SQ_VALU_MFMA_BUSY_CYCLES" for _, c in m) and any(c == "GRBM_GUI_ACTIVE" for _, c in m):
        print("\nderived (per dispatch): GRBM_GUI_ACTIVE is summed over the 8 XCDs (active_per_clk = GRBM_GUI_ACTIVE /\n"
              " (dispatch duration x 2.4 GHz) reads about 8, a little less when the clock runs below 2.4 GHz), so\n"
              " mfma_util = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 * 1024 SIMDs);\n"
              " flops = 512 * SQ_INSTS_VALU_MFMA_MOPS_<type>, TFLOP/s over the dispatch duration;\n"
              " lds_conflict = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE")
        print("kernel".ljust(56) + "mfma_util".rjust(12) + "f32_TFLOPs".rjust(12) + "bf16_TFLOPs".rjust(12) +
              "lds_conflict".rjust(14) + "active_per_clk".rjust(16))
        for kn in kernels:
            g = lambda c: m.get((kn, c), (None,))[0]
            busy, act = g("SQ_VALU_MFMA_BUSY_CYCLES"), g("GRBM_GUI_ACTIVE")
            util = f"{busy / (act / 8 * 1024):.4f}" if busy is not None and act else "-"
            f32 = g("SQ_INSTS_VALU_MFMA_MOPS_F32")
            bf = g("SQ_INSTS_VALU_MFMA_MOPS_BF16")
            conf, idx = g("SQ_LDS_BANK_CONFLICT"), g("SQ_LDS_IDX_ACTIVE")
            dur = g("duration_us")
            clk = f"{act / (dur * 1e-6 * 2.4e9):.2f}" if act and dur else "-"
            rate = lambda mops: "-" if mops is None or not dur else f"{512 * mops / (dur * 1e-6) / 1e12:.1f}"
            print(kn[:55].ljust(56) + util.rjust(12) + rate(f32).rjust(12) + rate(bf).rjust(12) +
                  (f"{conf / idx:.4f}" if conf is not None and idx else "-").rjust(14) + clk.rjust(16))


def stats_summary(paths):
    """rocprofv3 --stats kernel table: calls, mean/min/max duration (us), share of kernel time."""
    import csv
    rows = []
    for f in csv_files(paths, "kernel_stats.csv"):
        rows += list(csv.DictReader(open(f)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print("kernel".ljust(64) + "calls".rjust(7) + "avg_us".rjust(10) + "min_us".rjust(10) + "max_us".rjust(10) +
          "pct".rjust(7))
    for r in rows:
        print(short_kernel_name(r["Name"])[:63].ljust(64) + r["Calls"].rjust(7) +
              f"{float(r['AverageNs']) / 1e3:.2f}".rjust(10) + f"{float(r['MinNs']) / 1e3:.2f}".rjust(10) +
              f"{float(r['MaxNs']) / 1e3:.2f}".rjust(10) + f"{float(r['Percentage']):.2f}".rjust(7))


def trace_summary(paths):
    """rocprofv3 --kernel-trace table per kernel and launch grid (the same kernel at different batch sizes,
    e.g. the batched step and the plain per-pair leg, gets one line each): calls, mean/min/max duration
    (us), share of kernel time."""
    import csv
    acc = {}
    for f in csv_files(paths, "kernel_trace.csv"):
        for r in csv.DictReader(open(f)):
            g = "x".join(r[c] for c in ("Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"))
            acc.setdefault((short_kernel_name(r["Kernel_Name"]), g), []).append(
                (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in acc.values())
    print("kernel".ljust(58) + "grid".rjust(14) + "calls".rjust(7) + "avg_us".rjust(10) + "min_us".rjust(10) +
          "max_us".rjust(10) + "pct".rjust(7))
    for (kn, g), v in sorted(acc.items(), key=lambda kv: -sum(kv[1])):
        print(kn[:57].ljust(58) + g.rjust(14) + str(len(v)).rjust(7) + f"{sum(v) / len(v):.2f}".rjust(10) +
              f"{min(v):.2f}".rjust(10) + f"{max(v):.2f}".rjust(10) + f"{100 * sum(v) / total:.2f}".rjust(7))


def traffic_summary(fetch, write, copy_fetch, copy_write, copy_kib=262144.0):
    """HBM bytes per dispatch from FETCH_SIZE and WRITE_SIZE runs, each scaled by what the same counter
    reads for the plain copy of copy_kib KiB (the largest kernel of the copy runs)."""
    f, w = counter_means([fetch]), counter_means([write])
    cf, cw = counter_means([copy_fetch]), counter_means([copy_write])
    cfk = max(v[0] for (k, c), v in cf.items() if c == "FETCH_SIZE")
    cwk = max(v[0] for (k, c), v in cw.items() if c == "WRITE_SIZE")
    ff, fw = copy_kib / cfk, copy_kib / cwk
    print(f"calibration: copy of {copy_kib:.0f} KiB reads FETCH_SIZE {cfk:.1f} KiB -> fetch factor {ff:.3f}; "
          f"WRITE_SIZE {cwk:.1f} KiB -> write factor {fw:.3f}")
    print()
    kernels = sorted({k for k, _ in f} | {k for k, _ in w},
                     key=lambda k: -(f.get((k, "FETCH_SIZE"), (0,))[0] + w.get((k, "WRITE_SIZE"), (0,))[0]))
    print("kernel".ljust(52) + "FETCH_KiB".rjust(13) + "WRITE_KiB".rjust(13) + "read_MB".rjust(10) + "write_MB".rjust(10))
    for k in kernels:
        fk = f.get((k, "FETCH_SIZE"), (0.0,))[0]
        wk = w.get((k, "WRITE_SIZE"), (0.0,))[0]
        print(k[:51].ljust(52) + f"{fk:.1f}".rjust(13) + f"{wk:.1f}".rjust(13) +
              f"{fk * ff * 1024 / 1e6:.2f}".rjust(10) + f"{wk * fw * 1024 / 1e6:.2f}".rjust(10))


def main():
    args = parse()
    if args.pmc_summary:
        return pmc_summary(args.pmc_summary)
    if args.stats_summary:
        return stats_summary(args.stats_summary)
    if args.trace_summary:
        return trace_summary(args.trace_summary)
    if args.traffic_summary:
        return traffic_summary(*args.traffic_summary)
    if args.cache_dir:
        os.environ["FMAP_BENCH_CACHE"] = args.cache_dir
    if args.oracle_one_pair:
        return oracle_one_pair(args.workload)
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build runs the solve on a single device (asked for --gpus "
              f"{args.gpus}); pairs are independent, so several GPUs would each take a share of the batch.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2604_10377_amd import fmap as F

    dev = torch.device("cuda:0")
    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("copied 3 x 256 MiB", flush=True)
        return
    if args.workload == "ragged":
        return bench_ragged(args, F, dev)
    if args.workload == "overlap":
        return bench_overlap(args, F, dev)
    if args.workload == "gradfeat":
        return bench_gradfeat(args, F, dev)
    if args.workload == "vectorized":
        return bench_vectorized(args, F, dev)
    if args.workload == "multires":
        return bench_multires(args, F, dev)
    if args.bwd is None:
        args.bwd = "recompute" if args.workload == "large" else "stored"
    b = make_workload(args.workload)
    bf16 = b.phi_bf16 is not None
    P = b.pairs
    opts = SOLVE_OPTS.get(args.workload, {})
    subs = split_pairs(P, args.split)
    S = len(subs)

    def upload(sel):
        idx = list(sel) + [P + p for p in sel]
        if bf16:
            phi = torch.from_numpy(b.phi_bf16[idx].view(np.int16)).to(dev).view(torch.bfloat16)
            feat = torch.from_numpy(b.feat_bf16[idx].view(np.int16)).to(dev).view(torch.bfloat16)
        else:
            phi = torch.from_numpy(b.phi[idx]).to(dev)
            feat = torch.from_numpy(b.feat[idx]).to(dev)
        t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
        return (phi, t(b.mass[idx]), feat, t(b.evals_x[list(sel)]), t(b.evals_y[list(sel)]), t(b.lam[list(sel)]),
                None if b.dC is None else t(b.dC[list(sel)]))

    base = [upload(sel) for sel in subs]
    sets = [base] + [[tuple(None if x is None else x.clone() for x in inp) for inp in base] for _ in range(2)]
    fwd_only = b.dC is None  # the plain workload is a forward solve
    stream = torch.cuda.current_stream(dev)
    side = [torch.cuda.Stream(dev) for _ in range(S - 1)]
    steps = [SplitStep([Step(F, dev, sub_batch(b, len(sel)), inp, args.bwd, **opts) for sel, inp in zip(subs, st)],
                       side) for st in sets]

    if args.profile_steps:
        for i in range(args.profile_steps):
            steps[i % 3].run()
        torch.cuda.synchronize()
        print(f"profiled {args.profile_steps} eager steps of {b.name} ({S} sub-batches)", flush=True)
        return

    # warm-up (also JIT-free: the library is AOT compiled) and graph capture
    for s in steps:
        s.run()
    torch.cuda.synchronize()
    graphs = None
    if not args.no_graph:
        graphs = []
        for s in steps:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                s.run()
            graphs.append(g)
        torch.cuda.synchronize()
    replay = (lambda i: graphs[i % 3].replay()) if graphs else (lambda i: steps[i % 3].run())
    warm_up(replay, args)
    ms, step_stats = timed_steps(replay, args.steps, stream)
    # accuracy from one more replay of input set 0 into outputs first filled with NaN, so that every
    # checked value comes from the replayed step itself
    for st in steps[0].steps:
        st.C.fill_(float("nan"))
        st.dF.fill_(float("nan"))
    replay(0)
    torch.cuda.synchronize()
    acc = accuracy(b, steps[0], pairs=(0, P - 1))

    # per-phase average duration of the sub-batch kernels, each phase alone: K more steps launched eagerly,
    # the sub-batches one after the other on the launch stream (the host stays ahead of the device, so the
    # kernels run back to back), HIP events on that stream between the phases.  A phase's time includes the
    # cache state the previous phases leave, e.g. the write-back of the backward projection's output during
    # the next forward projection.  In the timed graph the sub-batches overlap, so these are the kernels'
    # own rates, not their shares of the step.  (Events inside a captured graph are not available here.)
    phases = ("project", "solve") if fwd_only else ("project", "solve", "solve_backward", "project_backward")
    rs = torch.cuda.current_stream(dev)
    nev = len(phases) * S
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(nev + 1)] for _ in range(args.steps)]
    for i in range(max(args.warmup, 1)):
        for st in steps[i % 3].steps:
            st.run()
    torch.cuda.synchronize()
    for i in range(args.steps):
        evs[i][0].record(rs)
        e = 1
        for st in steps[i % 3].steps:
            for name in phases:
                getattr(st, name)()
                evs[i][e].record(rs)
                e += 1
    torch.cuda.synchronize()
    phase_ms = {name: 0.0 for name in phases}
    for i in range(args.steps):
        e = 0
        for _ in range(S):
            for name in phases:
                phase_ms[name] += evs[i][e].elapsed_time(evs[i][e + 1]) / args.steps
                e += 1
    # costs and roofline of one sub-batch launch of each phase (the launches the step is made of)
    sub0 = sub_batch(b, len(subs[0]))
    costs = {nme: c for nme, c in phase_costs(sub0, bf16).items() if nme in phase_ms}
    peaks = {nme: matrix_peak(nme, b, bf16) for nme in costs}
    launch_ms = {nme: v / S for nme, v in phase_ms.items()}
    dom = max([nme for nme in ("project", "project_backward") if nme in phase_ms], key=lambda nme: phase_ms[nme])
    roof = roofline_entry(costs[dom][0], costs[dom][1], launch_ms[dom] * 1e-3, peaks[dom][0])
    roof["matrix_path"] = peaks[dom][1]
    roof["kernel"] = ("fmap_project (split-K partials + fixed-order reduce)" if dom == "project" else
                      "fmap_project_backward") + f", one launch = {len(subs[0])} pairs"
    tr = measured_traffic(dom, args.workload, len(subs[0]))
    roof["traffic"] = None if tr is None else tr["bytes"]
    if tr is not None:
        roof["traffic_detail"] = tr | {"algorithmic_bytes": round(costs[dom][1])}
    roof["phase_us"] = {k: round(v * 1e3, 2) for k, v in phase_ms.items()}
    roof["phase_timing"] = (f"K eager steps after the timed ones, the {S} sub-batches in sequence, HIP events "
                            "between phases; summed over sub-batches, mean over the K steps")
    full_costs = {nme: c for nme, c in phase_costs(b, bf16).items() if nme in phase_ms}
    t_roof = sum(max(f / (peaks[nme][0] * 1e12), by / (HBM_PEAK_GBS * 1e9)) for nme, (f, by) in full_costs.items())
    roof["step_roofline_us"] = round(t_roof * 1e6, 2)
    roof["step_frac"] = round(t_roof * 1e3 / ms, 4)
    step_bytes = sum(by for _, by in full_costs.values())
    roof["step_hbm_GBs"] = round(step_bytes / (ms * 1e-3) / 1e9, 1)

    vs_plain = None
    if not args.no_plain and not fwd_only:
        pv, pms, pstats, psteps = plain_leg(args, F, b, dev, base_full(b, dev, upload, P), opts)
        pacc = accuracy_plain(b, psteps, pairs=(0, P - 1))
        vs_plain = {"value": round(pv, 1), "unit": "solves/s", "ms_per_step": round(pms, 5), "step_ms": pstats,
                    "ratio": round((P / (ms * 1e-3)) / pv, 3), "accuracy_vs_oracle": pacc,
                    "path": "plain float32 GPU path: per-pair library calls, eager launches, no graph, no "
                            "sub-batches, factors stored"}
    cpu = None if (args.no_cpu_baseline or fwd_only) else cpu_baseline(b, args.cpu_seconds, args.workload)
    out = {
        "metric": "functional map solves/sec (fwd+bwd) at k=50,d=256,batch 32" if args.workload == "headline"
        else f"functional map solves/sec ({'fwd' if fwd_only else 'fwd+bwd'}), {b.name}",
        "value": round(P / (ms * 1e-3), 1),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "step_ms": step_stats,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "vs_plain": vs_plain,
        "dtype": "bf16-proj/f32" if bf16 else "f32",
        "data": "synthetic",
        "config": {"workload": b.name, "pairs": P, "n": b.n, "k": b.k, "d": b.d,
                   "mask": "resolvent" if b.mask == 1 else "laplacian", "lambda": float(b.lam[0]),
                   "backward": args.bwd, "graph": not args.no_graph, "sub_batches": S, **opts},
        "roofline": roof,
        "cpu_baseline": cpu,
        "accuracy_vs_oracle": acc,
    }
    if args.workload == "large":
        out["peak_hbm_bytes"] = int(torch.cuda.max_memory_allocated(dev))
    print(json.dumps(out), flush=True)


def base_full(b, dev, upload, P):
    """The whole batch as one [2P] upload (the plain leg's per-pair slices index it)."""
    return upload(list(range(P)))


if __name__ == "__main__":
    main()
