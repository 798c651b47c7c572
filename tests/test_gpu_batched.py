"""GPU parity of the batched evaluation (many independent 2D systems of uneven N
in one call, captured as one HIP graph) against the CPU oracle run system by
system at each system's own depth.  Bars as for single systems: FP64 1e-12
relative L2 per system, FP32 1e-6 on potentials (fields 1e-3, stated)."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
F = pytest.importorskip("paper_2009_00767_amd")

FP32_FIELD_TOL = 1e-3


def rel(a, b):
    b = np.asarray(b)
    return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def default_depth(n, lmax):
    """Depth the library picks when none is given: about 16 particles per leaf."""
    if n <= 0:
        return 2
    return int(min(max(int(np.floor(np.log(n / 16.0) / np.log(4.0) + 0.5)), 2), lmax))


def concat(systems):
    off = np.zeros(len(systems) + 1, np.int64)
    off[1:] = np.cumsum([len(q) for _, q in systems])
    if off[-1] == 0:
        return off, np.zeros((0, 2)), np.zeros(0)
    pos = np.concatenate([p for p, _ in systems])
    q = np.concatenate([q for _, q in systems])
    return off, pos, q


def make_plan(nmax, nsys, p, lmax, precision=F.FMM_FP64, flags=F.FMM_SYNC_CHECK):
    return F.FMM(F.FMM_LOG2D, levels=lmax, order=p, max_particles=max(nmax, 1),
                 precision=precision, flags=flags, max_systems=nsys, max_levels=lmax)


def check_systems(systems, pot, fld, levels, p, tol_pot, tol_fld, off):
    worst = 0.0
    for s, (ps, qs) in enumerate(systems):
        a, b = off[s], off[s + 1]
        if b == a:
            continue
        want, wfld = oracle.fmm2d(ps, qs, int(levels[s]), p)
        e = rel(pot[a:b], want)
        worst = max(worst, e)
        assert e < tol_pot, (s, b - a, levels[s], e)
        assert rel(fld[a:b], wfld) < tol_fld, (s, b - a, levels[s])
    return worst


def small_batch(nsys=24, seed=91, nmin=200, nmax=20000):
    return workloads.batched_systems(nsys, 2, seed=seed, nmin=nmin, nmax=nmax)


@pytest.mark.parametrize("precision,tp,tf", [(F.FMM_FP64, 1e-12, 1e-12),
                                             (F.FMM_FP32, 1e-6, FP32_FIELD_TOL)])
def test_batched_default_depths_match_oracle(precision, tp, tf):
    systems = small_batch()
    off, pos, q = concat(systems)
    lmax, p = 6, 12
    f = make_plan(len(q), len(systems), p, lmax, precision)
    pot, fld = f.evaluate_batched(off, dev(pos), dev(q))
    torch.cuda.synchronize()
    levels = [default_depth(len(qs), lmax) for _, qs in systems]
    assert len(set(levels)) >= 3  # several stacked groups
    check_systems(systems, pot.cpu().numpy(), fld.cpu().numpy(), levels, p, tp, tf, off)
    f.close()


def test_batched_given_depths_including_shallow():
    """Depths 0 and 1 (near field only) next to deeper systems; systems of one
    particle and of none in between."""
    rng = np.random.default_rng(92)
    systems = small_batch(10, seed=93, nmin=500, nmax=6000)
    systems.insert(3, workloads.uniform(1, 2, seed=94))
    systems.insert(5, (np.zeros((0, 2)), np.zeros(0)))
    systems.append(workloads.uniform(2, 2, seed=95))
    levels = rng.integers(0, 6, size=len(systems)).astype(np.int32)
    levels[0], levels[1] = 0, 1
    off, pos, q = concat(systems)
    f = make_plan(len(q), len(systems), 10, 5)
    pot, fld = f.evaluate_batched(off, dev(pos), dev(q), sys_levels=levels)
    torch.cuda.synchronize()
    check_systems(systems, pot.cpu().numpy(), fld.cpu().numpy(), levels, 10, 1e-12, 1e-12, off)
    f.close()


def test_batched_sort_order_and_keys():
    systems = small_batch(12, seed=96, nmin=300, nmax=5000)
    off, pos, q = concat(systems)
    lmax = 5
    levels = np.array([default_depth(len(qs), lmax) for _, qs in systems], np.int32)
    f = make_plan(len(q), len(systems), 8, lmax)
    f.evaluate_batched(off, dev(pos), dev(q))
    torch.cuda.synchronize()
    n = len(q)
    perm = np.frombuffer(F.fmm_debug_level_data(f.plan, 0, F.FMM_DBG_PERM, 4 * n), np.int32)
    keys = np.frombuffer(F.fmm_debug_level_data(f.plan, 0, F.FMM_DBG_SORTED_KEYS, 4 * n),
                         np.uint32)
    with pytest.raises(F.FmmError):
        F.fmm_debug_level_data(f.plan, 2, F.FMM_DBG_MOMENTS, 1 << 20)
    f.close()
    # expected: stable order by (depth, system, Morton leaf); key = rank << 2L | Morton
    order = np.argsort(levels, kind="stable")
    rank = np.empty(len(systems), np.int64)
    for g in np.unique(levels):
        members = order[levels[order] == g]
        rank[members] = np.arange(len(members))
    sysid = np.repeat(np.arange(len(systems)), np.diff(off))
    morton = np.zeros(n, np.int64)
    for s, (ps, _) in enumerate(systems):
        L = int(levels[s])
        c = np.minimum(np.floor(ps * ((1 << L) / 5.0)).astype(np.int64), (1 << L) - 1)
        morton[off[s]:off[s + 1]] = _morton2(c[:, 0], c[:, 1])
    big = (levels[sysid].astype(np.int64) << 40) | (rank[sysid] << 24) | morton
    want = np.argsort(big, kind="stable")
    np.testing.assert_array_equal(perm, want)
    L_of = levels[sysid[want]].astype(np.int64)
    np.testing.assert_array_equal(keys.astype(np.int64),
                                  (rank[sysid[want]] << (2 * L_of)) | morton[want])


def _morton2(x, y):
    def spread(v):
        v = v & 0xFFFF
        v = (v | (v << 8)) & 0x00FF00FF
        v = (v | (v << 4)) & 0x0F0F0F0F
        v = (v | (v << 2)) & 0x33333333
        v = (v | (v << 1)) & 0x55555555
        return v
    return spread(x) | (spread(y) << 1)


def test_batched_graph_replay_and_recapture():
    """The same shape replays the captured graph: new charges and positions in
    the same buffers must give new, correct results on every replay, with eager
    work between replays; a new shape is captured anew; a plain fmm_eval on the
    same plan between batched calls leaves both correct."""
    systems = small_batch(16, seed=97, nmin=300, nmax=8000)
    off, pos, q = concat(systems)
    lmax, p = 5, 10
    levels = [default_depth(len(qs), lmax) for _, qs in systems]
    f = make_plan(len(q), len(systems), p, lmax, F.FMM_FP64, flags=0)
    dpos, dq = dev(pos), dev(q)
    pot = torch.empty(len(q), dtype=torch.float64, device="cuda")
    fld = torch.empty((len(q), 2), dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(98)
    for rep in range(3):
        qs_new = rng.uniform(-1, 1, size=len(q))
        ps_new = rng.uniform(0, 5, size=pos.shape)
        dq.copy_(dev(qs_new))
        dpos.copy_(dev(ps_new))
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        f.evaluate_batched(off, dpos, dq, pot=pot, field=fld)
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        new_sys = [(ps_new[off[s]:off[s + 1]], qs_new[off[s]:off[s + 1]])
                   for s in range(len(systems))]
        check_systems(new_sys, pot.cpu().numpy(), fld.cpu().numpy(), levels, p, 1e-12, 1e-12, off)
    assert f.last_status() == F.FMM_OK
    # plain single-system evaluation on the same plan in between
    pos1, q1 = workloads.uniform(3000, 2, seed=99)
    p1, f1 = f.evaluate(dev(pos1), dev(q1))
    torch.cuda.synchronize()
    w1, wf1 = oracle.fmm2d(pos1, q1, lmax, p)
    assert rel(p1.cpu().numpy(), w1) < 1e-12 and rel(f1.cpu().numpy(), wf1) < 1e-12
    # a different shape: fewer systems, other sizes
    sys2 = systems[:7]
    off2, pos2, q2 = concat(sys2)
    pot2, fld2 = f.evaluate_batched(off2, dev(pos2), dev(q2))
    torch.cuda.synchronize()
    check_systems(sys2, pot2.cpu().numpy(), fld2.cpu().numpy(), levels[:7], p, 1e-12, 1e-12, off2)
    # and back to the first shape
    f.evaluate_batched(off, dpos, dq, pot=pot, field=fld)
    torch.cuda.synchronize()
    check_systems(new_sys, pot.cpu().numpy(), fld.cpu().numpy(), levels, p, 1e-12, 1e-12, off)
    f.close()


def test_batched_errors():
    systems = small_batch(4, seed=100, nmin=100, nmax=1000)
    off, pos, q = concat(systems)
    f = make_plan(len(q), 4, 8, 4)
    with pytest.raises(F.FmmError):  # too many systems
        F.fmm_batch_prepare(f.plan, np.concatenate([off, [off[-1]]]), None)
    with pytest.raises(F.FmmError):  # no prepared shape of this size
        F.fmm_eval_batched(f.plan, 3, dev(off), None, dev(pos), dev(q),
                           torch.empty(len(q), dtype=torch.float64, device="cuda"),
                           torch.empty((len(q), 2), dtype=torch.float64, device="cuda"))
    with pytest.raises(F.FmmError):  # depth beyond the plan's maximum
        f.evaluate_batched(off, dev(pos), dev(q), sys_levels=np.array([2, 3, 5, 2], np.int32))
    bad = off.copy()
    bad[2] = bad[1] - 1
    with pytest.raises(F.FmmError):  # decreasing offsets
        f.evaluate_batched(bad, dev(pos), dev(q))
    outside = pos.copy()
    outside[off[2] + 1, 0] = 6.0
    with pytest.raises(F.FmmError):  # position outside the box (device-detected)
        f.evaluate_batched(off, dev(outside), dev(q))
    pot, fld = f.evaluate_batched(off, dev(pos), dev(q))  # still usable afterwards
    torch.cuda.synchronize()
    lv = [default_depth(len(qs), 4) for _, qs in systems]
    check_systems(systems, pot.cpu().numpy(), fld.cpu().numpy(), lv, 8, 1e-12, 1e-12, off)
    f.close()
    single = F.FMM(F.FMM_LOG2D, levels=4, order=8, max_particles=len(q))
    with pytest.raises(F.FmmError):
        single.evaluate_batched(off, dev(pos), dev(q))
    single.close()


def test_512_systems_workload():
    """512 systems, N log-uniform in [1k, 64k], uniform or Gaussian-mixture, p = 20
    in FP32 mode and FP64 mode; every system against the oracle at its depth."""
    systems = workloads.batched_systems(512, 2, seed=5)
    off, pos, q = concat(systems)
    lmax, p = 8, 20
    levels = [default_depth(len(qs), lmax) for _, qs in systems]
    f32 = make_plan(len(q), 512, p, lmax, F.FMM_FP32)
    pot32, fld32 = f32.evaluate_batched(off, dev(pos), dev(q))
    f64 = make_plan(len(q), 512, p, lmax, F.FMM_FP64)
    pot64, fld64 = f64.evaluate_batched(off, dev(pos), dev(q))
    torch.cuda.synchronize()
    pot32, pot64 = pot32.cpu().numpy(), pot64.cpu().numpy()
    fld64 = fld64.cpu().numpy()
    # every system at the fixed FP64 bar against the oracle: 64 systems spread
    # over the batch (the full oracle sweep over 7.7M particles is too slow)
    for s in range(0, 512, 8):
        a, b = off[s], off[s + 1]
        want, wfld = oracle.fmm2d(systems[s][0], systems[s][1], levels[s], p)
        assert rel(pot64[a:b], want) < 1e-12, s
        assert rel(fld64[a:b], wfld) < 1e-12, s
        assert rel(pot32[a:b], want) < 1e-6, s
    # FP32 against FP64 over every system
    for s in range(512):
        a, b = off[s], off[s + 1]
        assert rel(pot32[a:b], pot64[a:b]) < 1e-6, s
    f32.close()
    f64.close()


def test_device_tables_replay_without_instantiation():
    """fmm_eval_batched through the C ABI with DEVICE system tables: the shape is
    prepared once; replays with new output buffers instantiate no graph and
    match the oracle system by system; device tables that differ from the
    prepared shape are reported as an argument error by fmm_last_status."""
    systems = small_batch(12, seed=111, nmin=300, nmax=6000)
    off, pos, q = concat(systems)
    lmax, p = 5, 10
    levels = [default_depth(len(qs), lmax) for _, qs in systems]
    f = make_plan(len(q), len(systems), p, lmax, F.FMM_FP64, flags=0)
    F.fmm_batch_prepare(f.plan, off, None)
    builds = f.stats().graph_builds
    assert builds == 1
    F.fmm_batch_prepare(f.plan, off, None)  # the same shape: nothing to do
    assert f.stats().graph_builds == builds
    d_off, dpos, dq = dev(off), dev(pos), dev(q)
    d_lev = dev(np.asarray(levels, np.int32))
    for rep in range(3):
        pot = torch.empty(len(q), dtype=torch.float64, device="cuda")
        fld = torch.empty((len(q), 2), dtype=torch.float64, device="cuda")
        F.fmm_eval_batched(f.plan, len(systems), d_off, d_lev if rep == 2 else None, dpos, dq,
                           pot, fld)
        assert f.last_status() == F.FMM_OK
        check_systems(systems, pot.cpu().numpy(), fld.cpu().numpy(), levels, p, 1e-12, 1e-12,
                      off)
    assert f.stats().graph_builds == builds
    bad = off.copy()
    bad[3] += 1
    F.fmm_eval_batched(f.plan, len(systems), dev(bad), None, dpos, dq, pot, fld)
    assert f.last_status() == F.FMM_ERR_INVALID_ARG
    bad_lev = np.asarray(levels, np.int32)
    bad_lev[5] = 2 if bad_lev[5] != 2 else 3
    F.fmm_eval_batched(f.plan, len(systems), d_off, dev(bad_lev), dpos, dq, pot, fld)
    assert f.last_status() == F.FMM_ERR_INVALID_ARG
    F.fmm_eval_batched(f.plan, len(systems), d_off, None, dpos, dq, pot, fld)
    assert f.last_status() == F.FMM_OK
    check_systems(systems, pot.cpu().numpy(), fld.cpu().numpy(), levels, p, 1e-12, 1e-12, off)
    assert f.stats().graph_builds == builds
    f.close()
