"""Temporal blocking and the autotuner, through the C ABI.

A blocked launch runs k iterations with the same per-point device code as
the single-step kernel, so blocked and single-step runs must agree bitwise:
states, waveform rows, across remainders (nsteps not a multiple of k), across
source batches (a block straddling a batch boundary), and at full size.  One
case is also checked against the oracle directly.  The autotuner must leave
the state, iteration count and source clock as they were, keep the fastest
pair, and serve a second context from its cache file.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import teuk_oracle as T
from paper_1001_3631_amd import workloads as W

from test_gpu_parity import SRC, STEP_GRIDS, gpu_engine, gpu_source, host, oracle_source, rel, to_dev

BLOCKS = [(4, 2), (8, 2), (4, 4)]


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1001_3631_amd import _lib
    _lib.load()


def run(grid, phi, pi, plan, src_amp=50.0):
    """plan = [((seg_rows, k_steps), nsteps), ...] run back to back from (phi, pi)
    with the synthetic source; returns (waveform, Phi, Pi) on the host."""
    total = sum(n for _, n in plan)
    eng = gpu_engine(grid)
    if phi is None:
        z = torch.zeros((grid["nth"], grid["nr"]), dtype=torch.complex128, device="cuda")
        eng.set_state(z, z)
    else:
        eng.set_state(to_dev(phi), to_dev(pi))
    gpu_source(eng, grid, dict(SRC, amplitude=src_amp), total)
    waves = []
    for (seg, k), n in plan:
        eng.set_tuning(seg, k)
        waves.append(host(eng.step(n)))
    p, q = eng.get_state()
    out = (np.concatenate(waves), host(p), host(q))
    assert eng.info["steps_done"] == total
    eng.close()
    return out


def assert_bitwise(a, b):
    for x, y in zip(a, b):
        assert x.shape == y.shape
        assert np.array_equal(x, y), float(np.max(np.abs(x - y)))


@pytest.mark.parametrize("block", BLOCKS, ids=lambda b: f"seg{b[0]}_k{b[1]}")
@pytest.mark.parametrize("gi", range(len(STEP_GRIDS)))
def test_block_bitwise_equal_to_single_iterations(gi, block):
    grid = STEP_GRIDS[gi]
    phi, pi = W.random_state(grid["nth"], grid["nr"], seed=13)
    ref = run(grid, phi, pi, [((4, 1), 11)])
    got = run(grid, phi, pi, [(block, 11)])      # 11 = blocks + a single-step remainder
    assert_bitwise(got, ref)


def test_block_against_oracle():
    grid = STEP_GRIDS[0]
    g = T.Grid(**grid)
    phi, pi = W.random_state(g.nth, g.nr, seed=17)
    w, p, q = run(grid, phi, pi, [((4, 4), 8)])
    src = oracle_source(g, dict(SRC, amplitude=50.0), 8)
    rp, rq = phi, pi
    rw = []
    for n in range(8):
        rp, rq = T.step(g, rp, rq, n, src)
        rw.append(rp[:, g.i_ext])
    assert rel(p, rp) <= 1e-13
    assert rel(q, rq) <= 1e-13
    assert rel(w, np.array(rw)) <= 1e-13


@pytest.mark.parametrize("lead", [1, 2, 3])
def test_block_straddling_a_source_batch(lead):
    """Source windows are produced 256 iterations at a time; after `lead`
    single iterations, blocks of 4 start at n = lead + 4j, and the one at
    252 + lead crosses the boundary at 256, so a new batch starts there (at
    253, 254 or 255)."""
    grid = STEP_GRIDS[0]
    phi, pi = W.random_state(grid["nth"], grid["nr"], seed=19)
    ref = run(grid, phi, pi, [((4, 1), 300)])
    got = run(grid, phi, pi, [((4, 1), lead), ((4, 4), 300 - lead)])
    assert_bitwise(got, ref)


@pytest.mark.parametrize("cfg", [W.KERR_EMRI, W.SCALE_GRID], ids=lambda c: c["name"])
def test_block_fullsize_bitwise(cfg):
    grid = cfg["grid"]
    ref = run(grid, None, None, [((8, 1), 24)], src_amp=1.0)
    assert np.max(np.abs(ref[1])) > 0.0
    for block in BLOCKS:
        got = run(grid, None, None, [(block, 24)], src_amp=1.0)
        assert_bitwise(got, ref)


def test_largest_grid_against_oracle():
    """The largest grid of the workloads (25600 x 512, the HBM-resident one,
    with its source): two iterations from a seeded random state as single
    steps at 16 rows and as one blocked (4, 2) launch (what the autotuner
    picks there) are bitwise equal, and match two oracle iterations at every
    point and in the waveform."""
    cfg = W.HBM_PLAIN
    grid = cfg["grid"]
    g = T.Grid(**grid)
    phi, pi = W.random_state(g.nth, g.nr, seed=91)
    outs = []
    for tuning in ((16, 1), (4, 2)):
        eng = gpu_engine(grid)
        eng.set_tuning(*tuning)
        gpu_source(eng, grid, cfg["source"], 4)
        eng.set_state(to_dev(phi), to_dev(pi))
        w = host(eng.step(2))
        outs.append((w,) + tuple(host(x) for x in eng.get_state()))
        eng.close()
    assert_bitwise(outs[1], outs[0])
    src = oracle_source(g, cfg["source"], 4)
    rp, rq, rw = T.evolve(g, phi, pi, 2, src)
    w, p, q = outs[0]
    e = (rel(p, rp), rel(q, rq), rel(w, rw))
    print("25600 x 512, two iterations against the oracle (Phi, Pi, waveform):", e)
    assert max(e) <= 1e-13, e


def test_invalid_tuning_is_rejected():
    from paper_1001_3631_amd._lib import TeukError
    eng = gpu_engine(STEP_GRIDS[0])
    before = eng.tuning
    for seg, k in ((16, 2), (4, 3), (12, 1), (8, 4), (4, 0)):
        with pytest.raises(TeukError):
            eng.set_tuning(seg, k)
    assert eng.tuning == before
    eng.close()


def test_autotune_with_source_keeps_the_evolution(tmp_path):
    """With an orbit table long enough for the trials the autotuner times
    with the source attached; afterwards the state, the iteration count and
    the source windows are as before: the evolution continues bit for bit
    as without the autotuner.  The cache key records the source."""
    grid = STEP_GRIDS[0]
    phi, pi = W.random_state(grid["nth"], grid["nr"], seed=24)
    n_orbit = 5 + 624 + 40
    outs = []
    for tune in (False, True):
        eng = gpu_engine(grid)
        eng.set_state(to_dev(phi), to_dev(pi))
        gpu_source(eng, grid, dict(SRC, amplitude=50.0), n_orbit)
        w0 = host(eng.step(5))
        if tune:
            cache = tmp_path / "tune_src.txt"
            table = eng.autotune(str(cache))
            assert len(table) == 3 + len(BLOCKS)
            assert "source=1" in cache.read_text()
            assert eng.info["steps_done"] == 5
        w1 = host(eng.step(30))
        outs.append((w0, w1) + tuple(host(x) for x in eng.get_state()))
        eng.close()
    assert_bitwise(outs[1], outs[0])


def test_autotune_keeps_state_and_serves_cache(tmp_path):
    grid = STEP_GRIDS[0]
    phi, pi = W.random_state(grid["nth"], grid["nr"], seed=23)
    cache = tmp_path / "tune.txt"

    eng = gpu_engine(grid)
    eng.set_state(to_dev(phi), to_dev(pi))
    gpu_source(eng, grid, dict(SRC, amplitude=50.0), 9)
    eng.step(5)
    before = tuple(host(x) for x in eng.get_state())
    table = eng.autotune(str(cache))
    assert len(table) == 3 + len(BLOCKS)
    assert {(s, k) for s, k, _ in table} == {(4, 1), (8, 1), (16, 1)} | set(BLOCKS)
    times = [us for _, _, us in table]
    assert all(t > 0.0 for t in times) and times == sorted(times)
    assert (eng.tuning["seg_rows"], eng.tuning["k_steps"]) == table[0][:2]
    assert eng.info["steps_done"] == 5
    assert_bitwise(tuple(host(x) for x in eng.get_state()), before)
    w_after = host(eng.step(4))
    p_after, q_after = (host(x) for x in eng.get_state())
    eng.close()

    ref = run(grid, phi, pi, [((4, 1), 5), ((4, 1), 4)])
    assert_bitwise((w_after, p_after, q_after), (ref[0][5:], ref[1], ref[2]))

    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].split("\t")[1:3] == [str(table[0][0]), str(table[0][1])]
    eng2 = gpu_engine(grid)
    hit = eng2.autotune(str(cache))
    assert len(hit) == 1 and hit[0][:2] == table[0][:2]
    assert (eng2.tuning["seg_rows"], eng2.tuning["k_steps"]) == table[0][:2]
    assert len(cache.read_text().splitlines()) == 1
    assert len(eng2.autotune(None)) == len(table)
    eng2.close()
