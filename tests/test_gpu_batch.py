"""Batched stepping through the C ABI, in both modes (one persistent graph
launch per call; one launch per iteration covering every instance).

Each instance of a batch must end bitwise equal to the same instance stepped
alone with teuk_step_n (same per-point device code): states and waveform rows,
for heterogeneous instances (a, m, s, grid shapes down to nr = 5, nth = 7,
dissipation on and off), for repeated launches of a cached graph, for a new
iteration count (new graph), for every segment length and both modes.  One instance is
also checked against the oracle directly, and the batched workload's real
shapes are covered by a subset of its instances.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import teuk_oracle as T
from paper_1001_3631_amd import workloads as W

from test_gpu_parity import SRC, STEP_GRIDS, gpu_engine, gpu_source, host, oracle_source, rel, to_dev


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1001_3631_amd import _lib
    _lib.load()


def make_batch(grids):
    from paper_1001_3631_amd.engine import Batch
    return Batch(grids)


def single_runs(grids, states, plan):
    """Each instance alone: plan = list of iteration counts run back to back."""
    out = []
    for g, (phi, pi) in zip(grids, states):
        eng = gpu_engine(g)
        eng.set_state(to_dev(phi), to_dev(pi))
        ws = [host(eng.step(n)) for n in plan]
        p, q = eng.get_state()
        out.append((np.concatenate(ws), host(p), host(q)))
        eng.close()
    return out


def batch_runs(grids, states, plan, seg=None, mode=None):
    b = make_batch(grids)
    if seg is not None:
        b.set_tuning(seg)
    if mode is not None:
        b.set_mode(mode)
        assert b.mode == mode
    for e, (phi, pi) in zip(b.instances, states):
        e.set_state(to_dev(phi), to_dev(pi))
    ws = [[] for _ in grids]
    for n in plan:
        w = b.step(n)
        for k in range(len(grids)):
            ws[k].append(host(w[k]))
    b.sync()
    out = []
    for k, e in enumerate(b.instances):
        p, q = e.get_state()
        out.append((np.concatenate(ws[k]), host(p), host(q)))
        assert e.info["steps_done"] == sum(plan)
    b.close()
    return out


def assert_bitwise(a, b):
    for x, y in zip(a, b):
        assert x.shape == y.shape
        assert np.array_equal(x, y), float(np.max(np.abs(x - y)))


MIXED = STEP_GRIDS + [
    dict(M=1.0, a=0.5, s=-1, m=3, nr=77, nth=33, rs_min=-30.0, rs_max=50.0, cfl=0.5, rs_extract=5.0, ko_eps=0.5),
]


MODES = [0, 1]   # Batch.PERSISTENT, Batch.PER_ITERATION


@pytest.mark.parametrize("mode", MODES, ids=["persistent", "per_iteration"])
@pytest.mark.parametrize("seg", [4, 8, 16])
def test_batch_bitwise_equal_to_single_instances(seg, mode):
    states = [W.random_state(g["nth"], g["nr"], seed=31 + k) for k, g in enumerate(MIXED)]
    plan = [5, 0, 5, 3]         # a cached graph replayed (after a call of no iterations), then a new count
    ref = single_runs(MIXED, states, plan)
    got = batch_runs(MIXED, states, plan, seg=seg, mode=mode)
    for a, b in zip(got, ref):
        assert_bitwise(a, b)


@pytest.mark.parametrize("mode", MODES, ids=["persistent", "per_iteration"])
def test_batch_instance_against_oracle(mode):
    grids = MIXED[:3]
    states = [W.random_state(g["nth"], g["nr"], seed=41 + k) for k, g in enumerate(grids)]
    got = batch_runs(grids, states, [4], mode=mode)
    for g_d, (phi, pi), (w, p, q) in zip(grids, states, got):
        g = T.Grid(**g_d)
        rp, rq = phi, pi
        rw = []
        for n in range(4):
            rp, rq = T.step(g, rp, rq, n, None)
            rw.append(rp[:, g.i_ext])
        assert rel(p, rp) <= 1e-13
        assert rel(q, rq) <= 1e-13
        assert rel(w, np.array(rw)) <= 1e-13


@pytest.mark.parametrize("mode", MODES, ids=["persistent", "per_iteration"])
def test_batched_workload_subset_bitwise(mode):
    """Instances of the batched workload at their real sizes (one of each grid
    level), Gaussian pulses, 12 iterations."""
    inst = W.batched_instances()
    pick = []
    for lvl in range(4):
        for it in inst:
            if it["grid"]["nth"] == 32 * 2 ** lvl:
                pick.append(it)
                break
    grids = [it["grid"] for it in pick]
    b = make_batch(grids)
    b.set_mode(mode)
    for e, it in zip(b.instances, pick):
        e.init_pulse(**it["pulse"])
    ws = b.step(12)
    b.sync()
    got = [(host(w),) + tuple(host(x) for x in e.get_state()) for w, e in zip(ws, b.instances)]
    b.close()
    for it, g_out in zip(pick, got):
        eng = gpu_engine(it["grid"])
        eng.init_pulse(**it["pulse"])
        w = host(eng.step(12))
        p, q = eng.get_state()
        assert_bitwise(g_out, (w, host(p), host(q)))
        assert np.max(np.abs(g_out[1])) > 0.0
        eng.close()


def test_batch_rejects_bad_arguments():
    from paper_1001_3631_amd._lib import TeukError
    grids = MIXED[:2]
    b = make_batch(grids)
    with pytest.raises(TeukError):
        b.set_tuning(12)
    assert b.mode == 1                 # the default: one launch per iteration
    with pytest.raises(TeukError):
        b.set_mode(2)
    assert b.mode == 1
    e = b.instances[0]
    orbit = e.orbit_circular(10.0, 9, M=1.0, a=grids[0]["a"])      # 4 iterations' worth of samples
    e.set_source(orbit, 1.0, 2.0, 2.0, 8.0)
    with pytest.raises(TeukError):                                 # ESTATE: orbit too short
        b.step(5)
    assert e.info["steps_done"] == 0 and b.instances[1].info["steps_done"] == 0
    assert e._lib.teuk_destroy(e.ctx) == -1        # TEUK_EINVAL: owned by the batch
    b.close()


# Sources in batched instances: every m of one orbit (a, grid shared), one
# instance on an inspiralling orbit table (r* of the circular orbit drifting
# inwards), and one without a source.
def _all_m_grids():
    base = dict(M=1.0, a=0.7, s=-2, nr=301, nth=33, rs_min=-40.0, rs_max=110.0, cfl=0.5, rs_extract=60.0,
                ko_eps=0.5)
    return [dict(base, m=m) for m in (1, 2, 3, 4)] + [dict(base, m=2), dict(base, m=3)]


def _orbits(engines, grids, nsamples):
    out = []
    for k, (e, g) in enumerate(zip(engines, grids)):
        if k == len(grids) - 1:
            out.append(None)                               # no source
            continue
        orb = e.orbit_circular(10.0, nsamples, M=g["M"], a=g["a"])
        if k == len(grids) - 2:                            # inspiralling table
            orb = orb.copy()
            orb[:, 0] -= 2e-3 * np.arange(nsamples)
        out.append(orb)
    return out


@pytest.mark.parametrize("mode", MODES, ids=["persistent", "per_iteration"])
def test_batch_with_sources_bitwise_equal_to_single_instances(mode):
    """300 iterations (two source batches) after 7 of instance 0 alone, so the
    instances' clocks differ; waveforms and states bitwise equal to each
    instance stepped alone with the same orbit."""
    grids = _all_m_grids()
    nsamples = 2 * 320 + 1
    states = [W.random_state(g["nth"], g["nr"], seed=61 + k) for k, g in enumerate(grids)]
    b = make_batch(grids)
    b.set_mode(mode)
    orbits = _orbits(b.instances, grids, nsamples)
    for e, (phi, pi), orb in zip(b.instances, states, orbits):
        e.set_state(to_dev(phi), to_dev(pi))
        if orb is not None:
            e.set_source(orb, 30.0, 2.0, 2.0, 8.0)
    pre = host(b.instances[0].step(7))
    ws = b.step(300)
    b.sync()
    got = [(host(w),) + tuple(host(x) for x in e.get_state()) for w, e in zip(ws, b.instances)]
    clocks = [e.info["steps_done"] for e in b.instances]
    b.close()
    assert clocks == [307] + [300] * (len(grids) - 1)
    for k, (g, (phi, pi), orb) in enumerate(zip(grids, states, orbits)):
        eng = gpu_engine(g)
        eng.set_state(to_dev(phi), to_dev(pi))
        if orb is not None:
            eng.set_source(orb, 30.0, 2.0, 2.0, 8.0)
        if k == 0:
            assert np.array_equal(host(eng.step(7)), pre)
        w = host(eng.step(300))
        p, q = eng.get_state()
        eng.close()
        assert_bitwise(got[k], (w, host(p), host(q)))
        assert np.max(np.abs(got[k][1])) > 0.0


# A batch whose two state levels exceed the last-level cache (256 MiB): the
# per-iteration mode packs its instances into groups of at most 96 MiB per
# level, first fit, largest first, held group by group in a device table
# whose order differs from the caller's.
def _level_bytes(g):
    return 2 * 16 * ((g["nr"] + 15) // 16 * 16) * g["nth"]


def _first_fit_decreasing(sizes, cap):
    bins, fill = [], []
    for k in sorted(range(len(sizes)), key=lambda k: -sizes[k]):
        for b in range(len(bins)):
            if fill[b] + sizes[k] <= cap:
                bins[b].append(k)
                fill[b] += sizes[k]
                break
        else:
            bins.append([k])
            fill.append(sizes[k])
    return [sorted(b) for b in bins]


def _cache_group_grids():
    base = dict(W.KERR_EMRI["grid"])
    return [dict(base, nr=801, nth=33, m=1),        # 0.9 MB per level
            dict(base, nr=6400, nth=256),           # 52 MB
            dict(base, nr=6400, nth=384),           # 79 MB
            dict(base, nr=12800, nth=256),          # 105 MB: beyond a group's 96 MiB, a group of its own
            dict(base, nr=3200, nth=128, m=3)]      # 13 MB


@pytest.mark.parametrize("mode", MODES, ids=["persistent", "per_iteration"])
def test_batch_in_cache_sized_groups_bitwise(mode):
    """The groups are the first-fit-decreasing packing of the instances'
    level sizes, and every instance (two with sources, 300 iterations: two
    source batches) ends bitwise equal to the same instance stepped alone."""
    grids = _cache_group_grids()
    sizes = [_level_bytes(g) for g in grids]
    assert 2 * sum(sizes) > 256 << 20
    expect = _first_fit_decreasing(sizes, 96 << 20)
    assert expect == [[3], [0, 2, 4], [1]]
    nsteps = 300
    states = [W.random_state(g["nth"], g["nr"], seed=81 + k) for k, g in enumerate(grids)]
    with_src = (0, 2)
    b = make_batch(grids)
    assert b.groups() == expect
    b.set_mode(mode)
    for k, (e, (phi, pi)) in enumerate(zip(b.instances, states)):
        e.set_state(to_dev(phi), to_dev(pi))
        if k in with_src:
            gpu_source(e, grids[k], SRC, nsteps)
    ws = b.step(nsteps)
    b.sync()
    got = [(host(w),) + tuple(host(x) for x in e.get_state()) for w, e in zip(ws, b.instances)]
    b.close()
    for k, (g, (phi, pi)) in enumerate(zip(grids, states)):
        eng = gpu_engine(g)
        eng.set_state(to_dev(phi), to_dev(pi))
        if k in with_src:
            gpu_source(eng, g, SRC, nsteps)
        w = host(eng.step(nsteps))
        p, q = eng.get_state()
        eng.close()
        assert_bitwise(got[k], (w, host(p), host(q)))
        assert np.max(np.abs(got[k][1])) > 0.0


def test_small_batch_is_one_group_in_the_callers_order():
    from paper_1001_3631_amd import _lib as L
    b = make_batch(MIXED)
    assert b.groups() == [list(range(len(MIXED)))]
    assert b._lib.teuk_batch_get_groups(b.ctx, None, None, None) == L.TEUK_EINVAL
    b.close()


@pytest.mark.parametrize("mode", MODES, ids=["persistent", "per_iteration"])
def test_batch_source_instance_against_oracle(mode):
    """An instance with a circular-orbit source, stepped in a batch, against
    the oracle directly (relative 1e-13)."""
    grids = [dict(M=1.0, a=0.6, s=-2, m=2, nr=200, nth=41, rs_min=-20.0, rs_max=40.0, cfl=0.5,
                  rs_extract=10.0, ko_eps=0.5), MIXED[1]]
    g = T.Grid(**grids[0])
    phi, pi = W.random_state(g.nth, g.nr, seed=71)
    b = make_batch(grids)
    b.set_mode(mode)
    e = b.instances[0]
    e.set_state(to_dev(phi), to_dev(pi))
    gpu_source(e, grids[0], dict(SRC, amplitude=50.0), 6)
    w = host(b.step(6)[0])
    b.sync()
    p, q = (host(x) for x in e.get_state())
    b.close()
    src = oracle_source(g, dict(SRC, amplitude=50.0), 6)
    rp, rq = phi, pi
    rw = []
    for n in range(6):
        rp, rq = T.step(g, rp, rq, n, src)
        rw.append(rp[:, g.i_ext])
    assert rel(p, rp) <= 1e-13
    assert rel(q, rq) <= 1e-13
    assert rel(w, np.array(rw)) <= 1e-13


@pytest.mark.parametrize("mode", MODES, ids=["persistent", "per_iteration"])
def test_all_m_workload_bitwise(mode):
    """The all-m batch at its real size (m = 1..4 of one orbit on 6400 x 128,
    each with the orbit's source), 12 iterations from pulses, bitwise equal to
    each instance stepped alone."""
    cfg = W.ALL_M
    src = cfg["source"]
    b = make_batch(cfg["grids"])
    b.set_mode(mode)
    orbits = []
    for e, g in zip(b.instances, cfg["grids"]):
        orb = e.orbit_circular(src["r0"], 2 * 12 + 1, M=g["M"], a=g["a"])
        orbits.append(orb)
        e.set_source(orb, 50.0, src["sigma_r_cells"], src["sigma_th_cells"], src["cutoff_sigmas"])
        e.init_pulse(50.0, 4.0, 1.0)
    ws = b.step(12)
    b.sync()
    got = [(host(w),) + tuple(host(x) for x in e.get_state()) for w, e in zip(ws, b.instances)]
    b.close()
    for g, orb, g_out in zip(cfg["grids"], orbits, got):
        eng = gpu_engine(g)
        eng.set_source(orb, 50.0, src["sigma_r_cells"], src["sigma_th_cells"], src["cutoff_sigmas"])
        eng.init_pulse(50.0, 4.0, 1.0)
        w = host(eng.step(12))
        p, q = eng.get_state()
        eng.close()
        assert_bitwise(g_out, (w, host(p), host(q)))
        assert np.max(np.abs(g_out[1])) > 0.0


def test_batch_autotune_restores_states(tmp_path):
    grids = MIXED[:4]
    states = [W.random_state(g["nth"], g["nr"], seed=51 + k) for k, g in enumerate(grids)]
    b = make_batch(grids)
    for e, (phi, pi) in zip(b.instances, states):
        e.set_state(to_dev(phi), to_dev(pi))
    b.step(3, waveform=False)
    before = [tuple(host(x) for x in e.get_state()) for e in b.instances]
    table = b.autotune(str(tmp_path / "tune.txt"))
    assert {(s, m) for s, m, _ in table} == {(s, m) for s in (4, 8, 16) for m in MODES}
    assert (b.seg_rows, b.mode) == table[0][:2]
    for e, st in zip(b.instances, before):
        assert_bitwise(tuple(host(x) for x in e.get_state()), st)
        assert e.info["steps_done"] == 3
    b.set_tuning(4 if table[0][0] != 4 else 8)
    b.set_mode(1 - table[0][1])
    hit = b.autotune(str(tmp_path / "tune.txt"))
    assert len(hit) == 1 and hit[0][:2] == table[0][:2]
    assert (b.seg_rows, b.mode) == table[0][:2]
    b.close()


def test_persistent_abort_is_reported_and_cleared():
    """The abort path of the persistent kernel, forced from the host: with the
    abort flag stored before the launch every wave leaves at its first pass,
    teuk_batch_sync reports TEUK_EDEVICE once and clears the flag, and the
    next launch on the same batch runs normally (bitwise equal to single
    instances)."""
    from paper_1001_3631_amd._lib import TEUK_EDEVICE, TeukError
    grids = MIXED[:3]
    states = [W.random_state(g["nth"], g["nr"], seed=71 + k) for k, g in enumerate(grids)]
    ref = single_runs(grids, states, [6])
    b = make_batch(grids)
    b.set_mode(0)
    for e, (phi, pi) in zip(b.instances, states):
        e.set_state(to_dev(phi), to_dev(pi))
    b.abort()
    b.step(6, waveform=False)
    with pytest.raises(TeukError) as ei:
        b.sync()
    assert ei.value.code == TEUK_EDEVICE
    b.sync()                                    # reported once, then cleared
    for e, (phi, pi) in zip(b.instances, states):
        e.set_state(to_dev(phi), to_dev(pi))
    w = b.step(6)
    b.sync()
    for k, e in enumerate(b.instances):
        p, q = e.get_state()
        assert_bitwise((host(w[k]), host(p), host(q)), ref[k])
    b.close()


def test_persistent_wait_limit_zero_ends_the_launch():
    """A zero wait limit makes every dependency wait that is not satisfied at
    its first check give up: the launch still ends (every wave leaves), and
    sync reports either a clean run or the abort.  With the default limit
    restored the batch runs normally again."""
    from paper_1001_3631_amd._lib import TEUK_EDEVICE, TeukError
    grids = [W.KERR_EMRI["grid"], MIXED[0]]
    states = [W.random_state(g["nth"], g["nr"], seed=81 + k) for k, g in enumerate(grids)]
    ref = single_runs(grids, states, [4])
    b = make_batch(grids)
    b.set_mode(0)
    for e, (phi, pi) in zip(b.instances, states):
        e.set_state(to_dev(phi), to_dev(pi))
    b.set_wait_limit(0.0)
    b.step(4, waveform=False)
    try:
        b.sync()
        print("zero wait limit: no wait gave up")
    except TeukError as ex:
        assert ex.code == TEUK_EDEVICE
        print("zero wait limit: abort reported")
    b.set_wait_limit(2.0)
    for e, (phi, pi) in zip(b.instances, states):
        e.set_state(to_dev(phi), to_dev(pi))
    w = b.step(4)
    b.sync()
    for k, e in enumerate(b.instances):
        p, q = e.get_state()
        assert_bitwise((host(w[k]), host(p), host(q)), ref[k])
    b.close()
