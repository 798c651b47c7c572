"""The multipole-to-local tile variants and their autotuner (2D and 3D):
every variant forms the same sums in the same order, so results must be
bit-identical; the tuner must pick a compiled variant, report its time and
reuse its choice for a plan of the same shape."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
F = pytest.importorskip("paper_2009_00767_amd")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


VARIANTS = [(1, 1), (1, 0), (2, 1), (2, 0), (3, 1), (4, 1), (4, 0), (8, 1), (8, 0)]


def overwrite(f, dpos, nq):
    """An evaluation with other charges, so that a box row a variant fails to
    write keeps a wrong value from it rather than the previous variant's
    (equal) one."""
    other = torch.from_numpy(np.random.default_rng(nq).uniform(-1, 1, nq)).cuda()
    f.evaluate(dpos, other)
    torch.cuda.synchronize()


@pytest.mark.parametrize("precision,p", [(F.FMM_FP32, 16), (F.FMM_FP32, 30), (F.FMM_FP64, 12),
                                         (F.FMM_FP64, 20), (F.FMM_FP64, 30),
                                         (F.FMM_BF16_M2L, 20)])
def test_every_variant_is_bit_identical(precision, p):
    pos, q = workloads.uniform(200000, 2, seed=701)
    L = 7
    f = F.FMM(F.FMM_LOG2D, levels=L, order=p, max_particles=len(q), precision=precision,
              flags=F.FMM_SYNC_CHECK)
    dpos, dq = dev(pos), dev(q)
    base = None
    ran = 0
    for mb, rm in VARIANTS:
        try:
            f.set_m2l_variant(mb, rm)
        except F.FmmError as e:
            assert e.status == F.FMM_ERR_INVALID_ARG  # not compiled for this precision / order
            continue
        overwrite(f, dpos, len(q))
        pot, fld = f.evaluate(dpos, dq)
        torch.cuda.synchronize()
        st = f.stats()
        assert (st.m2l_tile_mb, st.m2l_xcd_remap) == (mb, rm)
        if base is None:
            base = (pot.cpu().numpy(), fld.cpu().numpy())
        else:
            np.testing.assert_array_equal(pot.cpu().numpy(), base[0])
            np.testing.assert_array_equal(fld.cpu().numpy(), base[1])
        ran += 1
    f.close()
    assert ran >= 2


def test_autotuner_picks_and_caches():
    pos, q = workloads.uniform(1 << 20, 2, seed=2)
    opts = dict(levels=8, order=16, max_particles=len(q), precision=F.FMM_FP32,
                flags=F.FMM_AUTOTUNE)
    f = F.FMM(F.FMM_LOG2D, **opts)
    st = f.stats()
    assert st.m2l_tile_mb in (1, 2, 3, 4, 8) and st.m2l_xcd_remap in (0, 1)
    assert st.m2l_tuned_ms > 0
    pot, _ = f.evaluate(dev(pos), dev(q))
    g = F.FMM(F.FMM_LOG2D, **opts)  # same shape: the cached choice
    st2 = g.stats()
    assert (st2.m2l_tile_mb, st2.m2l_xcd_remap, st2.m2l_tuned_ms) == \
        (st.m2l_tile_mb, st.m2l_xcd_remap, st.m2l_tuned_ms)
    g.set_m2l_variant(1, 1)
    pot1, _ = g.evaluate(dev(pos), dev(q))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(pot.cpu().numpy(), pot1.cpu().numpy())
    print(f"tuned: tile_mb {st.m2l_tile_mb}, xcd_remap {st.m2l_xcd_remap}, "
          f"{st.m2l_tuned_ms:.4f} ms")
    f.close()
    g.close()
    h = F.FMM(F.FMM_COULOMB3D, levels=3, order=4, max_particles=10)
    for bad in ((3, 1), (2, 0), (0, 1), (4, 1)):  # (4: FP32 only)
        with pytest.raises(F.FmmError):
            h.set_m2l_variant(*bad)
    h.set_m2l_variant(2, 1)
    assert h.stats().m2l_tile_mb == 2
    h.close()


@pytest.mark.parametrize("precision,p,L", [(F.FMM_FP32, 8, 5), (F.FMM_FP32, 8, 3),
                                           (F.FMM_FP32, 4, 4), (F.FMM_FP32, 8, 6),
                                           (F.FMM_FP64, 8, 4), (F.FMM_FP64, 4, 3),
                                           (F.FMM_FP64, 8, 6)])
def test_3d_layers_per_wave_bit_identical(precision, p, L):
    """Two layers of 16 targets per wave, and (FP32) eight waves of two layers
    (workgroup blocks two and four times as deep, partly outside the grid at
    levels 3 and 4, fewer z blocks than x or y blocks from level 5) against one
    layer per wave; each variant after an evaluation with other charges."""
    pos, q = workloads.uniform(60000, 3, seed=702)
    f = F.FMM(F.FMM_COULOMB3D, levels=L, order=p, max_particles=len(q), precision=precision,
              flags=F.FMM_SYNC_CHECK)
    dpos, dq = dev(pos), dev(q)
    out = []
    for mb in ((1, 2, 4) if precision == F.FMM_FP32 else (1, 2)):
        f.set_m2l_variant(mb, 1)
        overwrite(f, dpos, len(q))
        pot, fld = f.evaluate(dpos, dq)
        torch.cuda.synchronize()
        assert f.stats().m2l_tile_mb == mb
        out.append((pot.cpu().numpy(), fld.cpu().numpy()))
    f.close()
    for o in out[1:]:
        np.testing.assert_array_equal(out[0][0], o[0])
        np.testing.assert_array_equal(out[0][1], o[1])


@pytest.mark.parametrize("L", [5, 6])
def test_3d_autotuner(L):
    """The tuned plan (whichever variant it chose) against the FP64 plan of the
    same shape, at levels where the variants number their blocks differently."""
    pos, q = workloads.uniform(1 << 18, 3, seed=703)
    f = F.FMM(F.FMM_COULOMB3D, levels=L, order=8, max_particles=len(q), precision=F.FMM_FP32,
              flags=F.FMM_AUTOTUNE | F.FMM_SYNC_CHECK)
    st = f.stats()
    assert st.m2l_tile_mb in (1, 2, 4) and st.m2l_xcd_remap == 1 and st.m2l_tuned_ms > 0
    dpos, dq = dev(pos), dev(q)
    pot, _ = f.evaluate(dpos, dq)
    torch.cuda.synchronize()
    f.close()
    g = F.FMM(F.FMM_COULOMB3D, levels=L, order=8, max_particles=len(q), precision=F.FMM_FP64,
              flags=F.FMM_SYNC_CHECK)
    ref, _ = g.evaluate(dpos, dq)
    torch.cuda.synchronize()
    g.close()
    ref = ref.cpu().numpy()
    err = np.linalg.norm(pot.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"level {L}: tuned tile_mb {st.m2l_tile_mb}, rel-L2 vs FP64 {err:.2e}")
    assert err < 1e-6


def test_autotune_cache_file(tmp_path):
    """With FMM_AUTOTUNE_CACHE set, a process writes its tuned variants to the
    JSON file, and a later process takes them from it instead of timing again
    (an edited time in the file comes back through fmm_get_stats)."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "m2l_tune.json"
    code = (f"import sys, json; sys.path.insert(0, {root!r})\n"
            "import paper_2009_00767_amd as F\n"
            "f = F.FMM(F.FMM_LOG2D, levels=7, order=16, precision=F.FMM_FP32, "
            "max_particles=1 << 16, flags=F.FMM_AUTOTUNE)\n"
            "s = f.stats()\n"
            "print(json.dumps([s.m2l_tile_mb, s.m2l_xcd_remap, s.m2l_tuned_ms]))\n")
    env = dict(os.environ, FMM_AUTOTUNE_CACHE=str(cache))

    def child():
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        return json.loads(r.stdout.strip().splitlines()[-1])

    mb, rm, ms = child()
    entries = json.loads(cache.read_text())["m2l_autotune"]
    assert len(entries) == 1
    e = entries[0]
    assert e["arch"] == "gfx950" and e["tile_mb"] == mb and e["xcd_remap"] == rm
    assert abs(e["ms"] - ms) < 1e-5 and e["key"][:3] == [2, 16, F.FMM_FP32]
    e["ms"] = 12.5  # a value no timing would give
    cache.write_text('{"m2l_autotune": [\n ' + json.dumps(e) + "\n]}\n")
    mb2, rm2, ms2 = child()
    assert (mb2, rm2) == (mb, rm) and abs(ms2 - 12.5) < 1e-6
