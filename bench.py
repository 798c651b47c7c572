#!/usr/bin/env python3
"""Throughput of the shift-free FMM on one MI355X.

One step = one full evaluation (bin and sort, moments at every level, the
interaction-list contraction at every level, local evaluation at every level,
near field, combine and unsort) of the benchmark workload, inputs resident in
HBM.  Prints ONE JSON line (see the fields below).

Default workload: 2D log kernel, N = 2^24 particles drawn from an
8-component Gaussian mixture (sigma 0.1, centres uniform in the 5 x 5 square),
charges uniform in [-1, 1], quadtree level 10, order 20: the largest
single-GPU configuration.  The mixed-precision (FP32) mode is timed and its
potentials are checked against the FP64 plain result (the metric is
particles/s at relative L2 error <= 1e-6 of the potential against that
result); the FP64 plain mode is timed beside it, and both are compared with the
direct sum at seeded sampled targets.  Other workloads (--workload) are the
named cases of the workloads module, among them the paper's own Section 3 runs
with its fixed point-charge box vectors.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particles/sec at rel-L2 1e-6 (mixed/learned vs FP64 plain); M2L MFMA %, P2P pairs/s"
PEAKS = {  # MI355X published dense peaks
    "hbm_GBs": 8000.0,
    "fp64_TFs": 78.6,
    "fp32_TFs": 157.3,
    "fp32_vector_TFs": 78.6,  # without packed FP32 instructions
    "bf16_TFs": 2500.0,
}
CU, LANES, CLOCK_GHZ = 256, 64, 2.4
# VALU instructions per near-field pair in the inner loops of the kernels' own
# gfx950 assembly, v_log_f32 / v_rcp_f32 / v_rsq_f32 counted once like any
# other (a bookkeeping peak: a register-only probe finds the transcendental
# instructions dearer than one slot, see the roofline note).  2D FP32: 10 in the
# direct kernel (80 in the body of its loop over eight sources), 12 in the
# LDS-tile kernel (whose per-source leaf offset costs two more); the lower
# count, i.e. the higher peak, is the one used.  2D FP64: 108 (software log and
# division); 3D FP32: 70 in the body of the loop over four sources; 3D FP64: 108
# in its loop over four (its r = 0 test a select, not a branch).
P2P_SLOTS = {(2, "fp32"): 10.0, (2, "fp64"): 108.0, (3, "fp32"): 17.5, (3, "fp64"): 27.0}


PHASE_STEPS = 5
CAL_BYTES = 64 << 20
COPY_BYTES = 1 << 30  # the known-size copy read and written once per run
# The paper's own runs of this method (Section 3, Tables 1-3: 3D, 4 x 4 x 4
# point charges per box, FP64 on an Intel Core i7-9700): N / total seconds.
# Another machine's figure, and its timed columns appear to leave out the near
# field: context for the ratio, not a target.
PAPER_PPS = {"3d-pm1-80k-L3-n4": 80000 / 9.4e-2, "3d-pm1-200k-L3-n4": 200000 / 1.1e-1,
             "3d-pm1-80k-L2-n4": 80000 / 1.4e-2}


def il_pairs(dim, L, lo=2):
    """Ordered (target, source) pairs over all interaction lists, levels lo..L.
    Per axis: 6n-8 index pairs have adjacent-or-equal parents, 3n-2 are adjacent."""
    tot = 0
    for k in range(max(lo, 2), L + 1):
        n = 1 << k
        tot += (6 * n - 8) ** dim - (3 * n - 2) ** dim
    return tot


def traffic_key(workload, levels_override, near, levels, root_frame, nodes, order=0):
    """The name a counter summary is filed under: the workload, and what was run
    on it other than its own tree and basis (adaptive depth, another deepest
    level, the root-frame passes, Chebyshev points)."""
    key = workload
    if near:
        key += f"-adaptive-L{levels}-T{near}"
    elif levels_override:
        key += f"-L{levels}"
    if root_frame:
        key += "-rootframe"
    if nodes != "paper":
        key += f"-{nodes}"
    if order:
        key += f"-order{order}"
    return key


def measured_traffic(workload, precision, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary of this
    configuration (profiles/traffic_<key>_<precision>.json, the key from
    traffic_key), or None when there is none or the kernel's sources changed since
    the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        table = json.load(fh)
    entry = table.get("kernels", {}).get(kernel)
    if entry is None:
        return None
    h = hashlib.sha256()
    for src in entry["sources"]:
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    return entry["hbm_bytes_per_launch"] if h.hexdigest() == entry["sha256"] else None


def p2p_pairs(pos, L, side=5.0):
    import numpy as np
    n, dim = pos.shape
    nl = 1 << L
    c = np.minimum(np.floor(pos * (nl / side)).astype(np.int64), nl - 1)
    lin = c[:, 0] + nl * c[:, 1] + (nl * nl * c[:, 2] if dim == 3 else 0)
    cnt = np.bincount(lin, minlength=nl ** dim).reshape((nl,) * dim)
    pad = np.pad(cnt, 1)
    nb = np.zeros_like(cnt)
    import itertools
    for off in itertools.product((0, 1, 2), repeat=dim):
        sl = tuple(slice(o, o + nl) for o in off)
        nb += pad[sl]
    return int((cnt * nb).sum() - n)


def adaptive_tree(pos, L, near, side=5.0):
    """Host-side depths and active boxes of the 2D adaptive tree (a particle's
    tree stops at the first level k >= 2 whose 3 x 3 boxes around its box hold
    at most `near` particles): returns (depth per particle, {k: per-box particle
    counts}, {k: 3 x 3 counts}, {k: active-box mask}) with row-major boxes."""
    import numpy as np
    nl = 1 << L
    lc = np.minimum(np.floor(pos * (nl / side)).astype(np.int64), nl - 1)
    cnt = {L: np.bincount(lc[:, 0] + nl * lc[:, 1], minlength=nl * nl).reshape(nl, nl)}
    for k in range(L - 1, 1, -1):
        c = cnt[k + 1]
        cnt[k] = c[0::2, 0::2] + c[1::2, 0::2] + c[0::2, 1::2] + c[1::2, 1::2]
    around = {}
    for k in range(2, L + 1):
        pad = np.pad(cnt[k], 1)
        m = cnt[k].shape[0]
        around[k] = sum(pad[1 + dy:1 + dy + m, 1 + dx:1 + dx + m]
                        for dy in (-1, 0, 1) for dx in (-1, 0, 1))
    dep = np.full(len(pos), L)
    open_ = np.ones(len(pos), bool)
    for k in range(2, L):
        b = lc >> (L - k)
        stop = open_ & (around[k][b[:, 1], b[:, 0]] <= near)
        dep[stop] = k
        open_ &= ~stop
    active = {2: np.ones_like(cnt[2], bool)}
    for k in range(3, L + 1):
        par = around[k - 1] > near
        active[k] = np.repeat(np.repeat(par, 2, axis=0), 2, axis=1)
    return dep, cnt, around, active, lc


def p2p_pairs_adaptive(pos, L, near):
    """Ordered near-field pairs of the adaptive tree: each particle against the
    particles of the 3 x 3 boxes around its box at its own depth."""
    dep, cnt, around, _, lc = adaptive_tree(pos, L, near)
    tot = 0
    for k in range(2, L + 1):
        m = dep == k
        b = lc[m] >> (L - k)
        tot += int(around[k][b[:, 1], b[:, 0]].sum()) - int(m.sum())
    return tot


def il_pairs_adaptive(pos, L, near, lo=2):
    """Interaction-list pairs of the active target boxes (whose parent's 3 x 3
    boxes hold more than `near` particles; every box at level 2), levels lo..L:
    |IL(b)| = 4 (in-grid boxes around the parent) - (in-grid boxes around b)."""
    import numpy as np
    _, _, _, active, _ = adaptive_tree(pos, L, near)
    tot = 0
    for k in range(max(lo, 2), L + 1):
        n = 1 << k
        i = np.arange(n)
        nbr = np.minimum(i + 1, n - 1) - np.maximum(i - 1, 0) + 1  # same-level, per axis
        pi = i >> 1
        pnb = np.minimum(pi + 1, n // 2 - 1) - np.maximum(pi - 1, 0) + 1  # parent level
        il = 4 * np.outer(pnb, pnb) - np.outer(nbr, nbr)
        tot += int(il[active[k]].sum())
    return tot


BATCHED = "2d-batched-512-p20"


def bench_batched(args):
    """512 independent 2D systems (N log-uniform in [1k, 64k], uniform or
    Gaussian mixture), one batched call per step (one HIP graph), learned
    per-level order in FP32 mode against the fixed order p = 20 in FP64."""
    import numpy as np
    import torch

    import paper_2009_00767_amd as F
    from paper_2009_00767_amd import order_model
    import workloads

    systems = workloads.batched_systems(512, 2, seed=5)
    off = np.zeros(len(systems) + 1, np.int64)
    off[1:] = np.cumsum([len(qs) for _, qs in systems])
    pos = np.concatenate([ps for ps, _ in systems])
    q = np.concatenate([qs for _, qs in systems])
    n = len(q)
    lmax = 8
    depths = [order_model.default_depth(len(qs), lmax) for _, qs in systems]
    dev = torch.device("cuda:0")
    dpos, dq = torch.from_numpy(pos).to(dev), torch.from_numpy(q).to(dev)
    prec_name = "fp32" if args.precision == "auto" else args.precision
    prec = {"fp64": F.FMM_FP64, "fp32": F.FMM_FP32, "bf16": F.FMM_BF16_M2L}[prec_name]

    def make(precision, learned, flags=0):
        f = F.FMM(F.FMM_LOG2D, levels=lmax, order=20, max_particles=n, precision=precision,
                  flags=flags | F.FMM_AUTOTUNE, max_systems=len(systems), max_levels=lmax,
                  tol=1e-6,
                  order_policy=F.FMM_ORDER_LEARNED if learned else F.FMM_ORDER_FIXED)
        if learned:
            f.set_order_model(order_model.load()[0])
        return f

    ref = make(F.FMM_FP64, False, F.FMM_SYNC_CHECK)
    ref_pot, _ = ref.evaluate_batched(off, dpos, dq)
    torch.cuda.synchronize()
    ref_pot = ref_pot.cpu().numpy()
    ref.close()

    fm = make(prec, True)
    pot = torch.empty(n, dtype=torch.float64, device=dev)
    fld = torch.empty((n, 2), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        fm.evaluate_batched(off, dpos, dq, stream=stream, pot=pot, field=fld)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        fm.evaluate_batched(off, dpos, dq, stream=stream, pot=pot, field=fld)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = max(wall * 1000.0, e0.elapsed_time(e1)) / args.steps
    st = fm.stats()
    status = fm.last_status()
    err = float(np.linalg.norm(pot.cpu().numpy() - ref_pot) / np.linalg.norm(ref_pot))
    fm.close()
    npairs = sum(p2p_pairs(ps, L) for (ps, _), L in zip(systems, depths))

    # What the learned order gains: the fixed order p = 20 in the same precision,
    # and the learned order with its judge (a fixed-order FP64 evaluation of the
    # same systems every call), timed the same way.
    def step_ms(f, steps):
        for _ in range(max(1, args.warmup // 2)):
            f.evaluate_batched(off, dpos, dq, stream=stream, pot=pot, field=fld)
        torch.cuda.synchronize()
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tw = time.perf_counter()
        c0.record(stream)
        for _ in range(steps):
            f.evaluate_batched(off, dpos, dq, stream=stream, pot=pot, field=fld)
        c1.record(stream)
        torch.cuda.synchronize()
        return max((time.perf_counter() - tw) * 1000.0, c0.elapsed_time(c1)) / steps

    fx = make(prec, False)
    fixed_ms = step_ms(fx, args.steps)
    fx.close()
    fj = make(prec, True, F.FMM_JUDGE)
    judged_ms = step_ms(fj, max(3, args.steps // 4))
    judge_status = fj.last_status()
    fj.close()
    # far-field work (interaction-list pairs x 8 (p_k + 1)^2 flop at each level's order)
    orders = list(st.order_per_level[:lmax + 1])
    work_fixed = work_learned = 0.0
    for L in depths:
        for k in range(2, L + 1):
            pairs = il_pairs(2, k, k)
            work_fixed += 8 * 21 ** 2 * pairs
            work_learned += 8 * (orders[k] + 1) ** 2 * pairs

    out = {
        "metric": METRIC, "value": n / (ms / 1e3), "unit": "particles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[prec_name],
        "data": "synthetic (seeded systems; no dataset)",
        "config": {"workload": BATCHED, "kernel": "log2d", "systems": len(systems), "n": n,
                   "depths": f"clamp(round(log4(N/16)), 2, {lmax}): "
                             f"{min(depths)}..{max(depths)}",
                   "order": "learned per level (fallback 20)", "precision": prec_name,
                   "orders_per_level": list(st.order_per_level[:lmax + 1]),
                   "rel_l2_pot_vs_fp64_fixed_p20": err, "meets_1e-6": err <= 1e-6,
                   "device_status": status, "near_pairs": npairs},
        "learned_vs_fixed": {
            "fixed_p20_ms": fixed_ms, "learned_ms": ms, "learned_with_judge_ms": judged_ms,
            "judge_status": judge_status,
            "far_field_work_learned_over_fixed": work_learned / work_fixed,
            "note": "same precision, stream and step count; FMM_JUDGE runs a fixed-order "
                    "FP64 evaluation of every system in each call and compares each "
                    "system's potentials; far-field work counts 8 (p_k + 1)^2 flop per "
                    "interaction-list pair at each level's order"},
        "roofline": None,
        "roofline_note": "one HIP graph per step: per-kernel durations come from the "
                         "rocprofv3 kernel trace, not from events",
    }
    print(json.dumps(out), flush=True)
    return 0


def host_cpu():
    """The host's CPU model and logical core count (nproc)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_sample_workload(w):
    """A bounded sample of a named workload for the oracle's timing: the same
    recipe and seed (for the mixture, the same centres) with the particle count
    divided by 2^D and the depth lowered by one, repeatedly, until at most 2^20
    particles remain (2^16 for the 3D harmonic expansions, whose oracle
    contraction costs 81 x 81 complex products per pair), so that the particles
    per leaf, the order and the distribution stay those of the workload."""
    import workloads
    n, L, dim = w["n"], w["levels"], w["dim"]
    cap = 1 << (16 if dim == 3 and w.get("basis") != "points" else 20)
    while n > cap and L > 2:
        n //= 1 << dim
        L -= 1
    if w["kind"] == "uniform":
        ps, qs = workloads.uniform(n, dim, w["seed"])
    elif w["kind"] == "pm1":
        ps, qs = workloads.plus_minus_one(n, dim, w["seed"])
    else:
        ps, qs = workloads.gaussian_mixture(n, dim, w["seed"])
    return ps, qs, L


def cpu_leg(args, w, pos, q, got, gotf, ref_pot, ref_fld, points, nodes="paper",
            root_frame=False, near=0):
    """The oracle's part of the run (CPU, FP64): the direct sum at seeded
    sampled targets, against which both GPU modes' potentials and fields are
    compared, and the oracle's own full evaluation timed on a bounded sample
    (median of three runs)."""
    import numpy as np

    import oracle
    import workloads

    n, dim, L, p = w["n"], w["dim"], w["levels"], w["p"]
    model, nproc = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", nproc))
    res = {}
    nt = args.direct_targets if args.direct_targets > 0 else (4096 if n <= (1 << 21) else 512)
    tg = workloads.sample_targets(n, nt, 1000 + w["seed"])
    t0 = time.perf_counter()
    dpot, dfld = oracle.direct(pos, q, targets=tg)
    td = time.perf_counter() - t0

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    res["vs_direct_sum"] = {
        "targets": int(len(tg)), "target_seed": 1000 + w["seed"],
        "rel_l2_pot_mode": rel(got[tg], dpot), "rel_l2_field_mode": rel(gotf[tg], dfld),
        "rel_l2_pot_fp64_plain": rel(ref_pot[tg], dpot),
        "rel_l2_field_fp64_plain": rel(ref_fld[tg], dfld),
        "oracle_seconds": td,
        "note": "the oracle's Neumaier-compensated FP64 direct sum over all particles at "
                "seeded sampled targets",
    }
    ps, qs, Ls = cpu_sample_workload(w)
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        if dim == 2 and near > 0:
            oracle.fmm2d_adaptive(ps, qs, Ls, p, near)
        elif dim == 2 and points:
            nd = oracle.chebyshev_nodes(p) if nodes == "chebyshev" else oracle.PAPER_NODES
            oracle.fmm2d_lagrange(ps, qs, Ls, nd)
        elif dim == 2:
            oracle.fmm2d(ps, qs, Ls, p)
        elif points:
            nd = oracle.chebyshev_nodes(p) if nodes == "chebyshev" else oracle.PAPER_NODES
            if root_frame:
                oracle.fmm3d_lagrange_root(ps, qs, Ls, nd)
            else:
                oracle.fmm3d_lagrange_nodes(ps, qs, Ls, nd)
        else:
            oracle.fmm3d(ps, qs, Ls, p)
        times.append(time.perf_counter() - t0)
    tc = float(np.median(times))
    res["cpu_baseline"] = {
        "value": len(qs) / tc, "unit": "particles/s", "cores": threads, "kind": "oracle",
        "sample": f"the oracle's full FP64 evaluation (level {Ls}, order {p}"
                  + (", root frame" if root_frame else "")
                  + (f", adaptive depth, 3 x 3 near field <= {near}" if near > 0 else "")
                  + f") of {len(qs)} "
                  f"particles drawn by the same recipe and seed as the workload"
                  + ("" if len(qs) == n else f" (N / {n // len(qs)}, level L - "
                     f"{L - Ls}: the same particles per leaf)")
                  + f"; median of 3 runs ({', '.join(f'{t:.2f}' for t in times)} s)",
        "host_cpu": model, "nproc": nproc, "omp_threads": threads,
    }
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="2d-mixture-16M-L10-p20")
    ap.add_argument("--precision", default="auto", choices=["auto", "fp64", "fp32", "bf16"])
    ap.add_argument("--nodes", default="paper", choices=["paper", "chebyshev"],
                    help="point-charge workloads: the paper's node set or Chebyshev points")
    ap.add_argument("--root-frame", action="store_true",
                    help="point-charge workloads: the root-frame passes (FP64)")
    ap.add_argument("--adaptive", type=int, default=0, metavar="T",
                    help="2D workloads: adaptive depth, a particle's tree stopping at the first "
                         "level whose 3 x 3 boxes around its box hold at most T particles")
    ap.add_argument("--levels", type=int, default=0,
                    help="deepest level (default: the workload's)")
    ap.add_argument("--order", type=int, default=0,
                    help="expansion order, or points per axis on the point-charge workloads "
                         "(Chebyshev points: 2..8 in 2D, 2..5 in 3D; default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--direct-targets", type=int, default=0,
                    help="sampled targets of the oracle's direct-sum check (0: 4096 up to 2^21 "
                         "particles, 512 above)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(the library runs on a single MI355X).",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2009_00767_amd as F
    import workloads

    if args.workload == BATCHED:
        return bench_batched(args)

    pos, q, w = workloads.make(args.workload)
    if args.levels > 0:
        w = dict(w, levels=args.levels)
    if args.order > 0:
        w = dict(w, p=args.order)
    n, dim, L, p = w["n"], w["dim"], w["levels"], w["p"]
    points = w.get("basis") == "points"
    near = args.adaptive
    if near and (dim != 2 or points or args.root_frame):
        print("--adaptive applies to the 2D workloads only", file=sys.stderr)
        return 2
    if (args.nodes != "paper" or args.root_frame) and not points:
        print("--nodes and --root-frame apply to the point-charge workloads only", file=sys.stderr)
        return 2
    if args.root_frame and dim != 3:
        print("--root-frame applies to the 3D point-charge workloads only", file=sys.stderr)
        return 2
    cheb = args.nodes == "chebyshev"
    if dim == 2:
        kernel = ((F.FMM_LOG2D_CHEBYSHEV if cheb else F.FMM_LOG2D_POINTS) if points
                  else F.FMM_LOG2D)
    else:
        kernel = ((F.FMM_COULOMB3D_CHEBYSHEV if cheb else F.FMM_COULOMB3D_POINTS) if points
                  else F.FMM_COULOMB3D)
    prec_name = args.precision
    if prec_name == "auto":
        prec_name = "fp64" if args.root_frame else "fp32"
    extra_flags = F.FMM_ROOT_FRAME if args.root_frame else 0
    prec = {"fp64": F.FMM_FP64, "fp32": F.FMM_FP32, "bf16": F.FMM_BF16_M2L}[prec_name]

    dev = torch.device("cuda:0")
    dpos = torch.from_numpy(pos).to(dev)
    dq = torch.from_numpy(q).to(dev)
    torch.cuda.synchronize()

    # FP64 plain reference result, and the FP64 plain mode's own step time
    # (a few evaluations after the first, same stream and event discipline).
    ref = F.FMM(kernel, levels=L, order=p, precision=F.FMM_FP64, max_particles=n,
                flags=F.FMM_SYNC_CHECK, adaptive_near=near)
    ref_pot, ref_fld = ref.evaluate(dpos, dq)
    torch.cuda.synchronize()
    ref_pot, ref_fld = ref_pot.cpu().numpy(), ref_fld.cpu().numpy()
    rpot = torch.empty(n, dtype=torch.float64, device=dev)
    rfld = torch.empty((n, dim), dtype=torch.float64, device=dev)
    fp64_steps = max(2, min(20, int(2e7 // n)))
    stream = torch.cuda.current_stream()
    ref.evaluate(dpos, dq, stream=stream, pot=rpot, field=rfld)
    torch.cuda.synchronize()
    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tw = time.perf_counter()
    r0.record(stream)
    for _ in range(fp64_steps):
        ref.evaluate(dpos, dq, stream=stream, pot=rpot, field=rfld)
    r1.record(stream)
    torch.cuda.synchronize()
    fp64_ms = max((time.perf_counter() - tw) * 1000.0, r0.elapsed_time(r1)) / fp64_steps
    ref.close()
    del rpot, rfld

    # Phase breakdown first, outside the timed region: a plan with an event at
    # every phase boundary (FMM_TIMING).  Its kernel times name the dominant
    # kernel; the timed plan then records events around that kernel's launch
    # only (each event record costs a few microseconds in its stream).
    def make(flags):
        return F.FMM(kernel, levels=L, order=p, precision=prec, max_particles=n,
                     flags=flags | F.FMM_AUTOTUNE | extra_flags, adaptive_near=near)

    try:
        fph = make(F.FMM_TIMING)
    except F.FmmError as e:
        if e.status != F.FMM_ERR_UNSUPPORTED or prec == F.FMM_FP64:
            raise
        prec_name, prec = "fp64", F.FMM_FP64
        fph = make(F.FMM_TIMING)
    pot = torch.empty(n, dtype=torch.float64, device=dev)
    fld = torch.empty((n, dim), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    for i in range(2 + PHASE_STEPS):
        fph.evaluate(dpos, dq, stream=stream, pot=pot, field=fld)
        if i == 1:
            torch.cuda.synchronize()
            fph.stats()
    torch.cuda.synchronize()
    sph = fph.stats()
    fph.close()
    # The main M2L's events in the phase plan also count the time it waits for
    # the chip while the near field runs beside it; the autotuner's timing of
    # the same launch alone decides which kernel dominates.
    # (adaptive depth: the tuner times the full grid; the phase plan's own launch,
    # which skips the inactive tiles, is the one to compare)
    m2l_alone = (sph.m2l_tuned_ms if sph.m2l_tuned_ms > 0 and not near
                 else sph.t_m2l_kernel_ms)
    dominant = "m2l" if m2l_alone > sph.t_p2p_ms else "p2p"

    fm = make(F.FMM_TIMING_M2L if dominant == "m2l" else F.FMM_TIMING_NEAR)
    for _ in range(args.warmup):
        fm.evaluate(dpos, dq, stream=stream, pot=pot, field=fld)
    torch.cuda.synchronize()
    fm.stats()  # reset the event ring: the averages below cover the timed steps only
    if fm.last_status() != F.FMM_OK:
        raise RuntimeError("device-detected error in warm-up")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        fm.evaluate(dpos, dq, stream=stream, pot=pot, field=fld)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    st = fm.stats()
    status = fm.last_status()
    ms = max(wall * 1000.0, ev_ms) / args.steps
    tuned = {"m2l_tile_mb": st.m2l_tile_mb, "m2l_xcd_remap": st.m2l_xcd_remap,
             "m2l_tuned_ms": st.m2l_tuned_ms}

    got = pot.cpu().numpy()
    gotf = fld.cpu().numpy()
    err_pot = float(np.linalg.norm(got - ref_pot) / np.linalg.norm(ref_pot))
    err_fld = float(np.linalg.norm(gotf - ref_fld) / np.linalg.norm(ref_fld))
    # the largest single-particle error, relative to the RMS of the reference
    rms_pot = float(np.linalg.norm(ref_pot)) / np.sqrt(n)
    rms_fld = float(np.linalg.norm(ref_fld)) / np.sqrt(n)
    maxe_pot = float(np.max(np.abs(got - ref_pot))) / rms_pot
    maxe_fld = float(np.max(np.linalg.norm(gotf - ref_fld, axis=1))) / rms_fld
    fm.close()

    # Algorithmic work per launch of the single-launch kernels, divided by that
    # kernel's own average duration (HIP events around the launch, on its stream).
    P = p + 1
    lo = st.m2l_kernel_level_lo
    npairs_il = il_pairs_adaptive(pos, L, near, lo) if near else il_pairs(dim, L, lo)
    # 2D: a complex P x P product; 3D: a real P^2 x P^2 one; point charges: a real
    # d x d one, d = n^2 (2D, n = p points per axis) or 64 (3D)
    if points:
        per_pair = 2 * (p * p) ** 2 if dim == 2 else 2 * 64 * 64
    else:
        per_pair = 8 * P * P if dim == 2 else 2 * P ** 4
    m2l_flops = per_pair * npairs_il
    npairs_p2p = p2p_pairs_adaptive(pos, L, near) if near else p2p_pairs(pos, L)
    phases = {"sort": sph.t_sort_ms, "p2m": sph.t_p2m_ms, "m2l": sph.t_m2l_ms,
              "l2p": sph.t_l2p_ms, "p2p": sph.t_p2p_ms}
    # the dominant kernel's time from the timed plan; the other M2L time is the
    # autotuner's (the launch alone), the other near-field time the phase plan's
    kernels = {"m2l": st.t_m2l_kernel_ms if dominant == "m2l" else m2l_alone,
               "p2p": st.t_p2p_ms if dominant == "p2p" else sph.t_p2p_ms}
    fp = prec_name
    tkey = traffic_key(args.workload, args.levels > 0, near, L, args.root_frame, args.nodes,
                       args.order)
    if dominant == "m2l":
        t = st.t_m2l_kernel_ms / 1e3
        peak = {"fp64": PEAKS["fp64_TFs"], "fp32": PEAKS["fp32_TFs"], "bf16": PEAKS["bf16_TFs"]}[fp]
        achieved = m2l_flops / t / 1e12
        roof = {"kernel": "m2l", "bound": "mfma", "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": measured_traffic(tkey, fp, "m2l"),
                "work_per_launch": f"{m2l_flops:.4e} flop = {per_pair} flop per interaction-list "
                                   f"pair x {npairs_il} pairs (levels {lo}..{L})",
                "launch_ms": st.t_m2l_kernel_ms}
    else:
        t = st.t_p2p_ms / 1e3
        slots = P2P_SLOTS[(dim, "fp64" if fp == "fp64" else "fp32")]
        peak = CU * LANES * CLOCK_GHZ * 1e9 / slots / 1e9
        achieved = npairs_p2p / t / 1e9
        roof = {"kernel": "p2p", "bound": "alu", "achieved": achieved, "peak": peak,
                "unit": "Gpair/s", "frac": achieved / peak,
                "traffic": measured_traffic(tkey, fp, "p2p"),
                "work_per_launch": f"{npairs_p2p} ordered near pairs; peak = 256 CU x 64 lanes "
                                   f"x 2.4 GHz / {slots} VALU issue slots per pair"
                                   + ("; the LDS-tile launch and the direct launch for tiles "
                                      "beyond its stage, timed together; a register-only issue "
                                      "probe of the direct kernel's pair (the same ten "
                                      "instructions, two of them transcendental) sustains "
                                      "3.44e12 pairs/s, 0.874 of this peak"
                                      if dim == 2 and fp != "fp64" else ""),
                "launch_ms": st.t_p2p_ms}

    # A plain copy of known size, for scaling the HBM byte counters of a profile run.
    cal_src = torch.empty(CAL_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    cal_dst = torch.empty_like(cal_src)
    cal_dst.copy_(cal_src)
    torch.cuda.synchronize()
    del cal_src, cal_dst
    # A bandwidth check of the HBM peak the roofline divides by: read + write
    # bytes of a 1 GiB elementwise copy (a kernel of its own, so that the 64 MiB
    # copy above stays the only copy a profile scales its counters by), the
    # fastest of six.
    big = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    big2 = torch.empty_like(big)
    best = 1e30
    for _ in range(6):
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        torch.mul(big, 1.0, out=big2)
        c1.record()
        torch.cuda.synchronize()
        best = min(best, c0.elapsed_time(c1))
    copy_gbs = 2 * COPY_BYTES / (best / 1e3) / 1e9
    del big, big2

    out = {
        "metric": METRIC,
        "value": n / (ms / 1e3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": (n / (ms / 1e3)) / PAPER_PPS[args.workload]
        if args.workload in PAPER_PPS else None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[fp],
        "data": "synthetic (seeded uniform positions, "
                + ("random +1/-1 charges" if w["kind"] == "pm1" else "charges in [-1, 1]")
                + "; no dataset)",
        "config": {"workload": args.workload,
                   "kernel": ("log2d" if dim == 2 else "coulomb3d")
                             + (f"_points_{args.nodes}" if points else ""),
                   "root_frame": bool(args.root_frame),
                   "tree": (f"adaptive depth: a particle's tree stops at the first level whose "
                            f"3 x 3 boxes around its box hold at most {near} particles, level "
                            f"{L} at most" if near else "uniform"),
                   "n": n, "levels": L, "order": p, "precision": fp,
                   "rel_l2_pot_vs_fp64_plain": err_pot, "rel_l2_field_vs_fp64_plain": err_fld,
                   "max_err_pot_over_rms": maxe_pot, "max_err_field_over_rms": maxe_fld,
                   "meets_1e-6": err_pot <= 1e-6,
                   "meets_1e-6_basis": "relative L2 error of the potential (the field's is "
                                       "stated beside it, not bounded)",
                   "field_meets_1e-6": err_fld <= 1e-6,
                   "device_status": status},
        "fp64_plain": {"ms_per_step": fp64_ms, "particles_per_s": n / (fp64_ms / 1e3),
                       "steps": fp64_steps},
        "m2l_autotune": tuned,
        "step_ms": {"wall_clock": wall * 1000.0 / args.steps, "hip_events": ev_ms / args.steps},
        "phases_ms": {k: round(v, 5) for k, v in phases.items()},
        "phase_total_ms": sph.t_total_ms,
        "phases_note": f"{PHASE_STEPS} evaluations before the timed ones, with an event at every "
                       "phase boundary; the near field overlaps the far-field phases; the timed "
                       "plan records events around the dominant kernel only",
        "kernels_ms": {k: round(v, 5) for k, v in kernels.items()},
        "kernels_note": "the dominant kernel from the timed plan's events; the main M2L otherwise "
                        "timed alone by the autotuner, the near field by the phase plan",
        "m2l_tflops": m2l_flops / (kernels["m2l"] / 1e3) / 1e12 if kernels["m2l"] > 0 else None,
        "p2p_pairs_per_s": npairs_p2p / (kernels["p2p"] / 1e3) if kernels["p2p"] > 0 else None,
        "roofline": roof,
        "hbm_copy_GBs": copy_gbs,
    }

    if not args.no_cpu_baseline:
        out.update(cpu_leg(args, w, pos, q, got, gotf, ref_pot, ref_fld, points,
                           args.nodes, args.root_frame, near))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
