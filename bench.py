"""Benchmark: particles/s per force evaluation of the periodic tree code on one
MI355X at the 1e-3 rms-force-error operating point.

Default workload: one GPU's share of the paper's run (Sec. 3: 10240^3
particles on ~1000 GPUs' worth of nodes), 1024^3 = 1,073,741,824 particles,
Zel'dovich displacements of a P(k) ~ k^-1.5 Gaussian field with rms
displacement 1.5 grid spacings, periodic unit box, order-4 multipoles, FP32
mixed precision, generated on the GPU.  One timed step = one kick-drift-kick
leapfrog step through the library (kick, drift with periodic wrap, one full
force evaluation: keys, sort, tree, moments, groups, walk, direct and
multipole interactions, far field, unpermute; kick).  Inputs are resident in
HBM before the timed region.

The operating point (acceptance-test tolerance and opening-angle cap) of each
workload is fixed in OPERATING_POINT; it was chosen by `--search` on one set
of targets, and the rms force error reported here is measured on a disjoint
held-out set: at 1024^3 against the FP64 GPU Ewald sum (libhotref), at 128^3
against the oracle's exact Ewald sum stored in tests/golden.

Beside the 1024^3 line the default run measures, at 128^3, the FP32/FP64
ratio of the force evaluation, the adjoint/forward ratio and the held-out
error, the differentiation workload (64^3, 10 checkpointed KDK steps), and
the oracle on the host's cores (cpu_baseline).

Prints one JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
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

METRIC = "particles/s per force eval at 1e-3 rms force err; FP32 vs FP64; adjoint/fwd"
FP32_PEAK_TFLOPS = 157.3      # MI355X dense FP32 vector (packed) peak
FP64_PEAK_TFLOPS = 78.6
ERR_TARGET = 1e-3
# --search keeps a margin below the target on its selection targets: the
# error on another set of targets (the held-out set the default run reports)
# differs by a few percent
SELECT_TARGET = 0.95 * ERR_TARGET

# The operating point of each workload: error-bound tolerance (absolute,
# acceleration units; the fraction of the workload's rms acceleration it was
# chosen as is noted), opening-angle cap, leaf and group sizes.  Chosen with
# --search on the selection targets; the error reported by a default run is
# measured on held-out targets that played no part in the choice.
OPERATING_POINT = {
    # 0.10 of a_rms = 0.0488, group-level local expansions of order 4 at
    # 0.003 of a_rms: selection error 9.35e-4 (without them the best
    # setting was 0.15 of a_rms at 9.08e-4 and 1.7x the time)
    "zeldovich128": dict(theta=0.8, err_tol=4.88e-3, leaf_max=16, group_max=128, local_order=4,
                         local_tol=1.46e-4),
    # 0.8 of a_rms = 34.4 with local expansions at 0.03 of a_rms: selection
    # error 9.40e-4 (without them 1.6 of a_rms at 8.92e-4 and 2x the time;
    # the clustered set's leaf/group sizes run faster at lower error: its
    # sparse background otherwise splits into many small groups)
    "nfw256": dict(theta=0.0, err_tol=34.4, leaf_max=32, group_max=256, local_order=4,
                   local_tol=1.29),
    # 0.09 of a_rms = 0.01857 with local expansions of order 4 at 0.008 of
    # a_rms: selection error 9.37e-4 (0.10 / 0.008: 9.88e-4, beyond the
    # search's margin, at 1.5% less time; without the local expansions 0.102
    # of a_rms, between the searched 0.09 at 8.06e-4 and 0.11 at 9.59e-4, at
    # 2.9x the time of the earlier local kernel); leaf 64 keeps the cells
    # within the 27-bit cell index of a list entry (the paper ends its
    # traversal below ~80 particles)
    "zeldovich1024": dict(theta=0.8, err_tol=1.67e-3, leaf_max=64, group_max=128, local_order=4,
                          local_tol=1.49e-4),
}
# --search grids: tolerances as fractions of the rms acceleration, opening-
# angle caps (0 = none), and opening angles alone
ETA_GRID = {"zeldovich128": (0.06, 0.08, 0.1, 0.12, 0.15, 0.18, 0.22, 0.27, 0.33),
            "nfw256": (0.8, 1.2, 1.6, 2.4, 3.5, 5.0, 7.0, 10.0),
            "zeldovich1024": (0.09, 0.10, 0.11, 0.12)}
THETA_CAPS = {"zeldovich128": (0.0, 0.7, 0.8, 0.9), "nfw256": (0.0, 0.8),
              "zeldovich1024": (0.8,)}
THETAS = {"zeldovich128": (0.40, 0.44, 0.46, 0.47, 0.48, 0.50), "nfw256": (0.3, 0.5, 0.7),
          "zeldovich1024": ()}
# group-level local expansions in the search: their order, and truncation
# tolerances as fractions of the rms acceleration (0 = none)
LOCAL_ORDER = 4
LOCAL_FRACS = {"zeldovich128": (0.0, 0.002, 0.003, 0.004, 0.005, 0.006),
               "nfw256": (0.0, 0.01, 0.03, 0.1, 0.2),
               "zeldovich1024": (0.004, 0.005, 0.0065, 0.008)}
# list region beside the minimum workspace at 1024^3 (the lists are processed
# in chunks of groups that fit it; 236 GB of workspace with the caller's 47 GB
# of arrays leave ~20 GB of the GPU's 288 GiB free)
PAPER_SCALE_LIST_BYTES = 32 << 30
# targets at 1024^3: 2000 distinct particles drawn with this seed, the first
# 1000 for --search (selection), the last 1000 for the reported error
C5_TARGET_SEED = 5
C5_TARGETS = 1000

WORKLOADS = {
    "zeldovich128": dict(
        ref="zeldovich128_ref.npz", heldout="zeldovich128_heldout.npz",
        data="synthetic (seeded Zel'dovich field standing in for the paper's 2LPT ICs)",
        desc="zeldovich {s}^3={n} particles, periodic unit box, P(k)~k^-1.5, rms displacement "
             "0.5 spacing"),
    "nfw256": dict(
        ref="nfw256_ref.npz", heldout=None,
        data="synthetic (seeded NFW halos, dN/dM~M^-1.9, c=8, plus uniform background, standing "
             "in for the paper's clustered late-time particle distributions)",
        desc="clustered {s}^3={n} particles: 70% in NFW halos of 1e2..1e5 particles, 30% "
             "uniform, periodic unit box"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="zeldovich1024",
                    choices=["zeldovich1024", "zeldovich128", "nfw256"],
                    help="zeldovich1024 (the headline: one GPU's share of the paper's run), "
                         "zeldovich128 or nfw256 (clustered)")
    ap.add_argument("--search", action="store_true",
                    help="search the operating point on the selection targets instead of using "
                         "OPERATING_POINT")
    ap.add_argument("--theta", type=float, default=None, help="override the opening-angle cap")
    ap.add_argument("--err-tol", type=float, default=None, help="override the tolerance")
    ap.add_argument("--leaf-max", type=int, default=None, help="override the leaf size")
    ap.add_argument("--group-max", type=int, default=None, help="override the sink-group size")
    ap.add_argument("--local-order", type=int, default=None,
                    help="override the order of the group-level local expansions (0 = none)")
    ap.add_argument("--local-tol", type=float, default=None,
                    help="override their truncation tolerance")
    ap.add_argument("--n-side", type=int, default=None, help="smaller grid (debug only)")
    ap.add_argument("--no-extras", action="store_true",
                    help="1024^3 run only: skip the 128^3 ratios and the trajectory adjoint")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-trajectory", action="store_true",
                    help="skip the differentiation-workload timing")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint timing (for profiling runs of the forward path)")
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--dt", type=float, default=0.01)
    ap.add_argument("--valu-probe", action="store_true",
                    help="only the vector-ALU throughput probe (the measured issue ceiling of the "
                         "force kernels' unpacked FP32 arithmetic)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only a plain 256 MiB device copy (three times), the reference the HBM "
                         "byte counters are scaled by")
    return ap.parse_args()


def copy_calibration():
    """A plain device copy of a known size: 256 MiB read and 256 MiB written
    per copy, three copies."""
    import torch
    x = torch.ones(64 * 2 ** 20, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": x.numel() * 4, "copies": 3}))


# HBM bytes of the dominant kernel per evaluation (the main and tail passes
# of every list chunk) from FETCH_SIZE/WRITE_SIZE counter runs, summarised in
# profiles/k_m2p_<workload>_hbm_counters.md.  Each holds only for the
# sources and the configuration it was taken with; otherwise the roofline
# reports traffic as null.
TRAFFIC_SOURCES = ["forces.hip", "device_math.h", "hot_internal.h", "walk.hip", "tree.hip"]
TRAFFIC = [
    {"workload": "zeldovich128", "kernel": "k_m2p<4,float>", "bytes_per_eval": 1.517e9,
     "config": {"theta": 0.8, "err_tol": 4.88e-3, "order": 4, "leaf_max": 16, "group_max": 128,
                "far_order": 8, "local_order": 4, "local_tol": 1.46e-4},
     "sha256": "b0569cd9b0c1a9885db49f54dcbc92e361477d32c8da0257d8e3a6a86b36d401"},
    {"workload": "zeldovich1024", "kernel": "k_m2p<4,float>", "bytes_per_eval": 3.910e11,
     "config": {"theta": 0.8, "err_tol": 1.67e-3, "order": 4, "leaf_max": 64, "group_max": 128,
                "far_order": 8, "local_order": 4, "local_tol": 1.49e-4},
     "sha256": "b0569cd9b0c1a9885db49f54dcbc92e361477d32c8da0257d8e3a6a86b36d401"},
]


def measured_traffic(prm, workload):
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1407_2600_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    for t in TRAFFIC:
        if workload == t["workload"] and h.hexdigest() == t["sha256"] and all(
                prm.get(k) == v for k, v in t["config"].items()):
            return t["bytes_per_eval"]
    return None


# Algorithmic HBM bytes of the bandwidth-bound stages (FP32 mode): the keys,
# sort and gather stage per particle (keys 36 B, 7 radix passes of 24 B,
# gather 56 B), and the build stage per particle and per cell (tree levels
# 12 B + 48 B/cell, moments and coefficient blocks 28 B + 600 B/cell, groups
# and source records 60 B).
SORT_BYTES_PER_PARTICLE = 36 + 7 * 24 + 56
BUILD_BYTES_PER_PARTICLE = 12 + 28 + 60
BUILD_BYTES_PER_CELL = 48 + 600


def stage_bandwidth(n, ncells, kern):
    """Achieved algorithmic GB/s of the sort and build stages against the
    8 TB/s HBM peak (both are one-pass streaming stages, several launches
    each, and at small sizes bound by launch latency rather than bytes)."""
    sort_b = SORT_BYTES_PER_PARTICLE * n
    build_b = BUILD_BYTES_PER_PARTICLE * n + BUILD_BYTES_PER_CELL * ncells
    out = {"unit": "GB/s", "peak": 8000.0}
    for name, b, ms in (("sort", sort_b, kern["ms_sort"]), ("build", build_b, kern["ms_build"])):
        gbs = b / (ms * 1e-3) / 1e9 if ms > 0 else None
        out[name] = {"bytes": b, "ms": ms, "achieved": gbs,
                     "frac": gbs / 8000.0 if gbs is not None else None}
    return out


def rms_err(a, ref):
    return float(np.sqrt(np.sum((a - ref) ** 2) / np.sum(ref ** 2)))


def max_err(a, ref):
    """Largest per-target force error over the rms reference acceleration."""
    d = np.sqrt(np.sum((a - ref) ** 2, axis=0))
    return float(np.max(d) / np.sqrt(np.mean(np.sum(ref ** 2, axis=0))))


def roofline(st, order, workload, prm):
    """The dominant force kernel (FP32): algorithmic flops of one evaluation
    over its HIP-event time (summed over the list chunks), against the FP32
    peak; and the other force kernels' rates."""
    names = {"m2p": f"k_m2p<{order},float>", "p2p": "k_p2p<float>",
             "m2l": f"k_m2l<{order},{prm.get('local_order', 0)},float>"}
    dom = max(("m2p", "p2p", "m2l"), key=lambda k: st[f"ms_{k}"])
    ms, fl = st[f"ms_{dom}"], st[f"flops_{dom}"]
    achieved = fl / (ms * 1e-3) / 1e12
    roof = {"kernel": names[dom],
            "bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": (measured_traffic(prm, workload) if dom == "m2p" and order == 4 else None),
            "flops_per_eval": fl, "ms_per_eval": ms, "launches_per_eval": st["list_chunks"]}
    ro = [{"kernel": names[k], "ms_per_eval": st[f"ms_{k}"],
           "achieved": (st[f"flops_{k}"] / (st[f"ms_{k}"] * 1e-3) / 1e12
                        if st[f"ms_{k}"] > 0 else None)}
          for k in ("m2p", "p2p", "m2l") if k != dom and st[f"ms_{k}"] > 0]
    return roof, ro


class StepStats:
    """Per-step sums of the library's stage times, pair counts and flops."""
    KEYS = ("ms_sort", "ms_build", "ms_walk", "ms_p2p", "ms_m2l", "ms_m2p", "ms_far", "ms_total")

    def __init__(self):
        self.k = {k: 0.0 for k in self.KEYS}
        self.pairs = {"p2p": 0.0, "m2p": 0.0, "m2l": 0.0}
        self.flops = {"p2p": 0.0, "m2p": 0.0, "m2l": 0.0}
        self.ncells = 0.0
        self.steps = 0
        self.last = None

    def add(self, st):
        for k in self.KEYS:
            self.k[k] += st[k]
        for q in ("p2p", "m2p", "m2l"):
            self.pairs[q] += st[f"{q}_pairs"]
            self.flops[q] += st[f"flops_{q}"]
        self.ncells += st["ncells"]
        self.steps += 1
        self.last = st

    def mean(self):
        s = max(self.steps, 1)
        st = dict(self.last)
        st.update({k: v / s for k, v in self.k.items()})
        for q in ("p2p", "m2p", "m2l"):
            st[f"{q}_pairs"] = self.pairs[q] / s
            st[f"flops_{q}"] = self.flops[q] / s
        st["ncells"] = self.ncells / s
        # lane use is taken from one step (its lane counters and its own
        # interactions): the steps' trees differ
        st["m2p_pairs_last"] = self.last["m2p_pairs"]
        return st


def pairs(st):
    """Interactions per evaluation: particle pairs of the direct kernel, and
    the particle-cell interactions taken by the multipole kernel and through
    the groups' local expansions (with the local-list entries that carry the
    latter)."""
    return {"p2p": st["p2p_pairs"], "m2p": st["m2p_pairs"], "m2l": st["m2l_pairs"],
            "m2l_entries": st["m2l_entries"]}


def lane_use(st):
    """Lane use of the multipole kernel: interactions over the lane-steps
    its main pass (64 lanes per pass of more than 32 targets) and tail pass
    (8, 16 or 32 lanes for a last pass of at most 32 targets) spend, per list
    entry, as counted by the library."""
    main, tail, tp = st["m2p_lanes_main"], st["m2p_lanes_tail"], st["m2p_pairs_tail"]
    mp = st.get("m2p_pairs_last", st["m2p_pairs"])
    if main + tail <= 0:
        return None
    return {"all": mp / (main + tail), "main": (mp - tp) / main if main else None,
            "tail": tp / tail if tail else None, "tail_pair_share": tp / mp if mp else None}


# the parameters --search chooses
SEARCHED = ("theta", "err_tol", "local_order", "local_tol")


def overrides(prm, args):
    """The operating point with the command line's overrides."""
    for k, a in (("theta", args.theta), ("err_tol", args.err_tol),
                 ("local_order", args.local_order), ("local_tol", args.local_tol),
                 ("leaf_max", args.leaf_max), ("group_max", args.group_max)):
        if a is not None:
            prm[k] = a
    return prm


def search(torch, Gravity, pos, mass, prm, tg, aref, dev, workload, **ctx):
    """The fastest setting of the searched grids whose FP32 rms force error
    on the selection targets tg is at most SELECT_TARGET."""
    a_rms = float(np.sqrt(np.mean(np.sum(aref ** 2, axis=0))))
    rows = []
    base = [dict(theta=cap, err_tol=float(f"{eta * a_rms:.3g}")) for cap in THETA_CAPS[workload]
            for eta in ETA_GRID[workload]]
    base += [dict(theta=th, err_tol=0.0) for th in THETAS[workload]]
    cands = [dict(b, local_order=LOCAL_ORDER if lf > 0 else 0,
                  local_tol=float(f"{lf * a_rms:.3g}") if lf > 0 else 0.0)
             for b in base for lf in LOCAL_FRACS[workload]]
    n = pos.shape[1]
    a = torch.empty((3, n), dtype=mass.dtype, device=dev)
    pt = torch.empty(n, dtype=mass.dtype, device=dev)
    for c in cands:
        g = Gravity(device=dev, **ctx, **dict(prm, **c))
        g.forces(pos, mass, out_acc=a, out_pot=pt)
        if "list_bytes" not in ctx:  # the second call runs with a sized workspace
            g.forces(pos, mass, out_acc=a, out_pot=pt)
        torch.cuda.synchronize()
        st = g.stats()
        e = rms_err(a[:, torch.as_tensor(tg, device=dev)].double().cpu().numpy(), aref)
        r = dict(c, err=e, ms_force=st["ms_total"], m2p_per_particle=st["m2p_pairs"] / st["n"],
                 p2p_per_particle=st["p2p_pairs"] / st["n"],
                 m2l_per_particle=st["m2l_pairs"] / st["n"], eta=c["err_tol"] / a_rms,
                 eta_local=c["local_tol"] / a_rms)
        rows.append(r)
        print(f"[bench] search {c} err={e:.3e} ms={st['ms_total']:.2f} "
              f"m2p/particle={r['m2p_per_particle']:.1f} p2p/particle={r['p2p_per_particle']:.1f} "
              f"local/particle={r['m2l_per_particle']:.1f}",
              file=sys.stderr, flush=True)
        del g
        torch.cuda.empty_cache()
    del a, pt
    torch.cuda.empty_cache()
    ok = [r for r in rows if r["err"] <= SELECT_TARGET]
    if not ok:
        raise SystemExit("no searched configuration reaches the target error")
    best = min(ok, key=lambda r: r["ms_force"])
    return best, rows


def paper_scale(args):
    """1024^3 Zel'dovich particles (rms displacement 1.5 spacings), one GPU's
    share of the paper's run: FP32 force evaluation and KDK steps at the
    fixed operating point, rms force error on held-out targets against the
    FP64 GPU Ewald sum."""
    import torch
    import workloads
    from paper_1407_2600_amd import Gravity
    from paper_1407_2600_amd.hotref import ewald_reference
    spec = workloads.WORKLOADS["zeldovich1024"]
    ns = args.n_side or spec["n_side"]
    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    pos = workloads.zeldovich_torch(ns, spec["seed"], rms_frac=spec["rms_frac"], device=dev)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    n = pos.shape[1]
    print(f"[bench] {n} particles generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    op = overrides(dict(OPERATING_POINT["zeldovich1024"]), args)
    prm = dict(box=1.0, G=1.0, eps=0.02 / ns, order=4, periodic=1, far_order=8,
               precision="fp32", **op)
    mass = torch.full((n,), 1.0 / n, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(C5_TARGET_SEED)
    draw = rng.choice(n, size=2 * C5_TARGETS, replace=False)
    select, held = np.sort(draw[:C5_TARGETS]), np.sort(draw[C5_TARGETS:])
    tg = select if args.search else held
    t0 = time.perf_counter()
    aref, _ = ewald_reference(pos, mass, tg, box=1.0, G=1.0, eps=prm["eps"])
    aref = aref.cpu().numpy()
    t_ref = time.perf_counter() - t0
    a_rms = float(np.sqrt(np.mean(np.sum(aref ** 2, axis=0))))
    print(f"[bench] FP64 Ewald reference on {len(tg)} targets in {t_ref:.1f} s, "
          f"rms |a| {a_rms:.4g}", file=sys.stderr, flush=True)
    ctx = dict(list_bytes=PAPER_SCALE_LIST_BYTES)
    found = None
    if args.search:
        best, rows = search(torch, Gravity, pos, mass, prm, tg, aref, dev, "zeldovich1024", **ctx)
        prm.update({k: best[k] for k in SEARCHED})
        found = {"chosen": best, "rows": rows, "targets": "selection"}
    g = Gravity(device=dev, **ctx, **prm)
    acc = torch.empty((3, n), dtype=torch.float32, device=dev)
    pot = torch.empty(n, dtype=torch.float32, device=dev)
    g.forces(pos, mass, out_acc=acc, out_pot=pot)
    torch.cuda.synchronize()
    st0 = g.stats()
    a_t = acc[:, torch.as_tensor(tg, device=dev)].double().cpu().numpy()
    err, emax = rms_err(a_t, aref), max_err(a_t, aref)
    print(f"[bench] force evaluation {st0['ms_total']:.0f} ms, rms error {err:.3e} "
          f"(max {emax:.3e}) on {'selection' if args.search else 'held-out'} targets",
          file=sys.stderr, flush=True)
    vel = torch.zeros((3, n), dtype=torch.float32, device=dev)
    for i in range(args.warmup):
        g.kdk(pos, vel, mass, acc, args.dt, 1, acc_valid=True, pot=pot, snapshot=False)
        print(f"[bench] warmup step {i}", file=sys.stderr, flush=True)
    ss = StepStats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        g.kdk(pos, vel, mass, acc, args.dt, 1, acc_valid=True, pot=pot, snapshot=False)
        ss.add(g.stats())  # this step's force evaluation (HIP events)
        print(f"[bench] step {i}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / max(args.steps, 1)
    st = ss.mean()
    roof, roof_other = roofline(st, 4, "zeldovich1024", prm)
    out = {
        "metric": METRIC, "value": n / el, "unit": "particles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded Zel'dovich field generated on the GPU, standing in for the "
                "paper's 10240^3 initial conditions; one GPU's share)",
        "config": {"workload": f"zeldovich {ns}^3={n} particles, periodic unit box, "
                               "P(k)~k^-1.5, rms displacement 1.5 spacing",
                   "theta": prm["theta"], "err_tol": prm["err_tol"], "order": 4,
                   "leaf_max": prm["leaf_max"], "group_max": prm["group_max"], "far_order": 8,
                   "eps": prm["eps"], "local_order": prm.get("local_order", 0),
                   "local_tol": prm.get("local_tol", 0.0),
                   "step": "one KDK step (one force evaluation), no state snapshots"},
        "rms_force_err": {"value": err, "max_over_rms": emax, "targets": len(tg),
                          "target_set": "selection" if args.search else "held-out",
                          "reference": "FP64 Ewald sum on the GPU (libhotref), rms |a| "
                                       f"{a_rms:.5g}", "reference_s": t_ref},
        "per_force_eval": {"fp32_ms": st0["ms_total"], "fp32_pps": n / (1e-3 * st0["ms_total"])},
        "stage_ms": {k: st[k] for k in StepStats.KEYS},
        "pairs_per_step": pairs(st),
        "m2p_lane_use": lane_use(st),
        "stage_bandwidth": stage_bandwidth(n, st["ncells"], st),
        "interactions_per_s": (st["p2p_pairs"] + st["m2p_pairs"] + st["m2l_pairs"]) / el,
        "list_chunks": st["list_chunks"], "workspace_bytes": int(g.ws.numel()),
        "roofline": roof, "roofline_other": roof_other,
        "operating_point_search": found,
    }
    del g, acc, pot, vel, pos, mass
    torch.cuda.empty_cache()
    return out


def load_refs(workload):
    W = WORKLOADS[workload]
    R = np.load(os.path.join(ROOT, "tests", "golden", W["ref"]))
    out = {"select": (R["targets"], R["acc_near_far"])}
    if W["heldout"]:
        H = np.load(os.path.join(ROOT, "tests", "golden", W["heldout"]))
        out["heldout"] = (H["targets"], H["acc_ewald"])
    return out


def workload_rates(args, workload, kdk_steps=True, adjoint=True):
    """One of the CPU-referenced workloads (128^3 Zel'dovich, 256^3 clustered)
    at its fixed operating point: FP32 and FP64 force evaluations (HIP-event
    medians), errors on the selection and held-out targets, the adjoint
    against the forward, and optionally timed KDK steps."""
    import torch
    import workloads
    from paper_1407_2600_amd import Gravity
    W = WORKLOADS[workload]
    pos_np, mass_np, prm = workloads.make(workload, n_side=args.n_side)
    prm = overrides(dict(prm, **OPERATING_POINT[workload]), args)
    n = pos_np.shape[1]
    dev = torch.device("cuda", 0)
    pos_dev = torch.as_tensor(pos_np, dtype=torch.float64, device=dev).contiguous()
    refs = load_refs(workload) if args.n_side is None else {}
    found = None
    if args.search and "select" in refs:
        m32 = torch.as_tensor(mass_np, dtype=torch.float32, device=dev)
        best, rows = search(torch, Gravity, pos_dev, m32, dict(prm, precision="fp32"),
                            refs["select"][0], refs["select"][1], dev, workload)
        prm.update({k: best[k] for k in SEARCHED})
        found = {"chosen": best, "rows": rows, "targets": "selection"}
    res = {}
    for prec in ("fp32", "fp64"):
        g = Gravity(device=dev, precision=prec, **prm)
        dt_ = torch.float32 if prec == "fp32" else torch.float64
        pos = pos_dev.clone()
        mass = torch.as_tensor(mass_np, dtype=dt_, device=dev)
        a0, p0 = g.forces(pos, mass)
        a0, p0 = g.forces(pos, mass)
        torch.cuda.synchronize()
        a_first = a0.double().cpu().numpy()
        f_ms, st = [], None
        for _ in range(5):
            g.forces(pos, mass, out_acc=a0, out_pot=p0)
            st = g.stats()
            f_ms.append(st["ms_total"])
        r = {"ms_force": float(np.median(f_ms)), "pps_force": n / (1e-3 * float(np.median(f_ms))),
             "stats": st, "workspace_bytes": int(g.ws.numel()), "errors": {}}
        for name, (tg, aref) in refs.items():
            r["errors"][name] = {"rms": rms_err(a_first[:, tg], aref),
                                 "max_over_rms": max_err(a_first[:, tg], aref), "targets": len(tg)}
        if prec == "fp32" and adjoint and not args.no_adjoint:
            # the adjoint is built without the group-level local route: the
            # ratio is taken at the same acceptance test with both routes off
            g_fwd = g
            if prm.get("local_order", 0) and prm.get("local_tol", 0.0):
                g = Gravity(device=dev, precision=prec, **dict(prm, local_order=0))
                g.forces(pos, mass, out_acc=a0, out_pot=p0)
            gen = torch.Generator(device=dev).manual_seed(7)
            gacc = torch.randn((3, n), dtype=dt_, device=dev, generator=gen)
            gpot = torch.randn(n, dtype=dt_, device=dev, generator=gen)
            # as autograd's backward runs it (after the forward at the same
            # point, on that evaluation's tree and lists), and with its own
            # tree build (hot_vjp)
            ta, tb, tf = [], [], []
            for rep in range(4):
                g.forces(pos, mass, out_acc=a0, out_pot=p0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g.vjp(pos, mass, gacc, gpot, after_forces=True)
                torch.cuda.synchronize()
                if rep:
                    ta.append(time.perf_counter() - t0)
            for rep in range(4):
                t0 = time.perf_counter()
                g.vjp(pos, mass, gacc, gpot)
                torch.cuda.synchronize()
                if rep:
                    tb.append(time.perf_counter() - t0)
            for rep in range(4):
                t0 = time.perf_counter()
                g.forces(pos, mass, out_acc=a0, out_pot=p0)
                torch.cuda.synchronize()
                if rep:
                    tf.append(time.perf_counter() - t0)
            adj = {"ms_vjp": 1e3 * float(np.median(ta)), "ms_forward": 1e3 * float(np.median(tf)),
                   "vjp_reuses_forward_tree": True,
                   "ms_vjp_with_tree_build": 1e3 * float(np.median(tb))}
            adj["ratio"] = adj["ms_vjp"] / adj["ms_forward"]
            adj["ratio_with_tree_build"] = adj["ms_vjp_with_tree_build"] / adj["ms_forward"]
            adj["local_expansions"] = bool(g is g_fwd and prm.get("local_order", 0))
            r["adjoint"] = adj
            if g is not g_fwd:
                del g
                g = g_fwd
                g.forces(pos, mass, out_acc=a0, out_pot=p0)
        if kdk_steps:
            vel = torch.zeros((3, n), dtype=dt_, device=dev)
            acc = a0.clone()
            pot = p0.clone()
            for _ in range(args.warmup):
                g.kdk(pos, vel, mass, acc, args.dt, 1, acc_valid=True, pot=pot)
            ss = StepStats()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                g.kdk(pos, vel, mass, acc, args.dt, 1, acc_valid=True, pot=pot)
                ss.add(g.stats())
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            r["kdk"] = {"steps": args.steps, "ms_per_step": 1e3 * el / max(args.steps, 1),
                        "pps": n * args.steps / el, "stats": ss.mean()}
        print(f"[bench] {workload} {prec}: force {r['ms_force']:.2f} ms, errors {r['errors']}",
              file=sys.stderr, flush=True)
        res[prec] = r
        del g
        torch.cuda.empty_cache()
    return n, prm, res, found


def extras_128(args):
    """The 128^3 keys of the default line: FP32/FP64, adjoint/forward and the
    held-out error of the force evaluation at its operating point, with the
    multipole kernel's roofline there (where its HBM counters were taken)."""
    n, prm, res, _ = workload_rates(args, "zeldovich128", kdk_steps=False)
    r32, r64 = res["fp32"], res["fp64"]
    roof, roof_other = roofline(r32["stats"], prm["order"], "zeldovich128", prm)
    return {
        "workload": WORKLOADS["zeldovich128"]["desc"].format(s=128, n=n),
        "config": {k: prm.get(k, 0) for k in ("theta", "err_tol", "order", "leaf_max",
                                              "group_max", "far_order", "eps", "local_order",
                                              "local_tol")},
        "fp32_ms": r32["ms_force"], "fp64_ms": r64["ms_force"],
        "fp32_pps": r32["pps_force"], "fp64_pps": r64["pps_force"],
        "fp32_over_fp64": r32["pps_force"] / r64["pps_force"],
        "rms_force_err": {"fp32": r32["errors"], "fp64": r64["errors"],
                          "heldout_reference": "oracle's exact Ewald sum on 1024 held-out "
                                               "targets",
                          "select_reference": "oracle's theta=0 near+far sum on the 10^4 "
                                              "selection targets"},
        "adjoint": r32.get("adjoint"),
        "adjoint_over_forward": r32["adjoint"]["ratio"] if "adjoint" in r32 else None,
        "stage_ms": {k: r32["stats"][k] for k in StepStats.KEYS},
        "m2p_lane_use": lane_use(r32["stats"]),
        "roofline": roof, "roofline_other": roof_other,
    }


def workload_main(args):
    """--workload zeldovich128 / nfw256: the line for that workload (FP32
    KDK steps as the headline value, FP64 beside it)."""
    n, prm, res, found = workload_rates(args, args.workload)
    r32, r64 = res["fp32"], res["fp64"]
    st = r32["kdk"]["stats"]
    roof, roof_other = roofline(st, prm["order"], args.workload, prm)
    W = WORKLOADS[args.workload]
    out = {
        "metric": METRIC, "value": r32["kdk"]["pps"], "unit": "particles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r32["kdk"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": W["data"],
        "config": {"workload": W["desc"].format(s=round(n ** (1 / 3)), n=n),
                   **{k: prm.get(k, 0) for k in ("theta", "err_tol", "order", "eps", "leaf_max",
                                                 "group_max", "far_order", "local_order",
                                                 "local_tol")},
                   "step": "one KDK step (one force evaluation)"},
        "rms_force_err": {"fp32": r32["errors"], "fp64": r64["errors"]},
        "per_force_eval": {"fp32_ms": r32["ms_force"], "fp32_pps": r32["pps_force"],
                           "fp64_ms": r64["ms_force"], "fp64_pps": r64["pps_force"]},
        "fp64": {"value": r64["kdk"]["pps"], "ms_per_step": r64["kdk"]["ms_per_step"],
                 "dtype": "f64"},
        "fp32_over_fp64": r32["pps_force"] / r64["pps_force"],
        "adjoint_over_forward": r32["adjoint"]["ratio"] if "adjoint" in r32 else None,
        "adjoint": r32.get("adjoint"),
        "interactions_per_s": ((st["p2p_pairs"] + st["m2p_pairs"] + st["m2l_pairs"]) /
                               (st["ms_total"] * 1e-3)),
        "stage_ms": {k: st[k] for k in StepStats.KEYS},
        "stage_bandwidth": stage_bandwidth(n, st["ncells"], st),
        "pairs_per_step": pairs(st),
        "m2p_lane_use": lane_use(st),
        "workspace_bytes": {"fp32": r32["workspace_bytes"], "fp64": r64["workspace_bytes"]},
        "roofline": roof, "roofline_other": roof_other,
        "operating_point_search": found,
    }
    if args.workload == "zeldovich128" and args.n_side is None and not args.no_trajectory:
        import torch
        dev = torch.device("cuda", 0)
        out["trajectory_adjoint"] = {p: trajectory_adjoint(torch, dev, p) for p in ("fp32", "fp64")}
    out["cpu_baseline"] = (None if args.no_cpu_baseline or args.n_side is not None
                           else cpu_baseline(args.cpu_seconds))
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_calibration:
        return copy_calibration()
    if args.valu_probe:
        from paper_1407_2600_amd.hotref import valu_probe
        r = valu_probe()
        for v in r.values():
            # per SIMD (1024 on the chip) per ns; unpacked FP32 lane-flops of an fma
            v["per_simd_per_ns"] = v["wave_instr_per_s"] / 1024 / 1e9
        print(json.dumps({"valu_probe": r}))
        return
    if args.workload != "zeldovich1024":
        print(json.dumps(workload_main(args)))
        return
    out = paper_scale(args)
    if not args.no_extras:
        import torch
        ex = extras_128(argparse.Namespace(**dict(vars(args), n_side=None, theta=None,
                                                  err_tol=None, search=False)))
        out["fp32_over_fp64"] = ex["fp32_over_fp64"]
        out["adjoint_over_forward"] = ex["adjoint_over_forward"]
        if not args.no_trajectory:
            dev = torch.device("cuda", 0)
            ex["trajectory_adjoint"] = {p: trajectory_adjoint(torch, dev, p)
                                        for p in ("fp32", "fp64")}
            print(f"[bench] trajectory adjoint {ex['trajectory_adjoint']}", file=sys.stderr,
                  flush=True)
            # the differentiation workload's backward/forward beside the
            # single-evaluation ratio (it is above 3 in FP64)
            out["trajectory_backward_over_forward"] = {
                p: ex["trajectory_adjoint"][p]["backward_over_forward"] for p in ("fp32", "fp64")}
        out["at_128cubed"] = ex
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline(args.cpu_seconds)
    print(json.dumps(out))


def trajectory_adjoint(torch, dev, precision="fp64", nsteps=10, dt=0.01):
    """The differentiation workload: 64^3 Zel'dovich particles at rest, 10
    KDK steps with per-step checkpoints, loss = sum of squared minimum-image
    distances to a second seed's end state; forward and backward times."""
    import workloads
    from paper_1407_2600_amd import Gravity, checkpointed_kdk
    pos, mass, prm = workloads.make("adjoint64")
    pos_t, _, _ = workloads.make("adjoint64", seed=workloads.WORKLOADS["adjoint64"]["seed"] + 100)
    g = Gravity(device=dev, precision=precision, **prm)
    dt_ = torch.float32 if precision == "fp32" else torch.float64
    M = torch.as_tensor(mass, dtype=dt_, device=dev)
    V0 = torch.zeros((3, pos.shape[1]), dtype=dt_, device=dev)
    with torch.no_grad():
        xt, _ = checkpointed_kdk(g, torch.as_tensor(pos_t, device=dev), V0, M, dt, nsteps)
    L = float(prm["box"])
    times = []
    for _ in range(2):  # the first round sizes the workspace
        P = torch.as_tensor(pos, device=dev).requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xf, _ = checkpointed_kdk(g, P, V0, M, dt, nsteps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        d = xf - xt
        d = d - L * torch.round(d / L)
        (d * d).sum().backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times.append((t1 - t0, t2 - t1))
    fwd, bwd = times[-1]
    return {"workload": f"zeldovich 64^3={pos.shape[1]} particles at rest, {nsteps} KDK steps "
                        f"dt={dt}, theta={prm['theta']}, order {prm['order']}, "
                        "per-step position checkpoints",
            "precision": precision, "ms_forward": 1e3 * fwd, "ms_backward": 1e3 * bwd,
            "backward_over_forward": bwd / fwd}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _omp_threads(k):
    """Set the OpenMP thread count of this process's runtime (the oracle's)."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(k))
        return True
    except OSError:
        return False


def cpu_baseline(seconds):
    """The oracle (FP64 same-test tree, plain C + OpenMP over sink groups) on
    the host's cores at the 128^3 Zel'dovich workload and its operating point
    (the 1024^3 set has the same recipe; its oracle tree would need more than
    150 GB of host memory): the full tree build plus forces for an evenly
    spaced sample of sink groups, scaled to particles/s of a whole force
    evaluation; once on all cores and once on one core.  Beside it, full
    evaluations of the 16^3 workload (median of 3 after one warm-up)."""
    import oracle
    import workloads
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    pos, mass, prm = workloads.make("zeldovich128")
    prm = dict(prm, **OPERATING_POINT["zeldovich128"])
    n = pos.shape[1]

    def sampled(secs, ncal):
        t0 = time.perf_counter()
        T = oracle.Tree(pos, mass, dict(prm))
        t_build = time.perf_counter() - t0
        ng = oracle.lib().or_tree_ngroups(T.h)
        g0 = np.arange(0, ng, max(1, ng // ncal))[:ncal]
        t0 = time.perf_counter()
        _, p = T.forces(groups=g0)
        t_cal = time.perf_counter() - t0
        k0 = int(np.sum(~np.isnan(p)))
        per_group = k0 / max(len(g0), 1)
        want = int(max(16, (k0 / max(t_cal, 1e-9)) * secs / max(per_group, 1)))
        sel = np.arange(0, ng, max(1, ng // want))[:want]
        t0 = time.perf_counter()
        _, p = T.forces(groups=sel)
        t_f = time.perf_counter() - t0
        k = int(np.sum(~np.isnan(p)))
        del T
        rate = 1.0 / (t_f / k + t_build / n)
        return rate, (f"full tree build ({t_build:.1f} s for {n} particles) + forces for {k} "
                      f"targets in {len(sel)} evenly spaced sink groups ({t_f:.1f} s)")

    def c1_full():
        p1, m1, q1 = workloads.make("lattice16")
        ts = []
        for rep in range(4):
            t0 = time.perf_counter()
            oracle.Tree(p1, m1, q1).forces()
            if rep:
                ts.append(time.perf_counter() - t0)
        return {"particles": p1.shape[1], "median_s": float(np.median(ts)),
                "value": p1.shape[1] / float(np.median(ts))}

    rate, desc = sampled(seconds, 64)
    c1 = c1_full()
    one = None
    if _omp_threads(1):
        r1, d1 = sampled(seconds / 2, 8)
        one = {"value": r1, "cores": 1, "sample": d1, "c1_full": c1_full()}
        _omp_threads(threads)
    return {"value": rate, "unit": "particles/s", "cores": threads, "kind": "oracle",
            "sample": f"128^3 Zel'dovich at its operating point: {desc}; rate = 1 / (force time "
                      "per target + build time per particle)",
            "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "c1_full": c1, "one_core": one}


if __name__ == "__main__":
    main()
