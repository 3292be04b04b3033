"""Write the oracle fixtures that the full-run GPU parity tests compare against.

TEST INFRASTRUCTURE.  Every value stored here comes from the CPU FP64 oracle
(`oracle/teuk_oracle.py`); the inputs come from the seeded workload
descriptions (`paper_1001_3631_amd/workloads.py`, which holds no arithmetic of
the method).  Nothing here touches the HIP library.

The full fields of the large workloads are too big to keep, so each fixture
holds a sample of the final state that the GPU test compares element by
element:
  * whole theta rows: the poles and their neighbours, rows on the segment
    seams of the stencil's launch configurations, the equator;
  * whole r* columns: the radial ends' neighbours, strip seams (62-column
    strips), the extraction column, the columns around the source;
  * a seeded uniform sample of interior points;
  * the L2 norm of every row of Phi and Pi of the full state (so an error
    anywhere in a row moves that row's norm);
  * the waveform (Phi at the extraction column) after every `stride`-th
    iteration, and its global norm;
  * for source-driven fields that are still local (the eccentric-orbit
    workload after its first iterations), the whole rectangle around the
    particle.

Each workload has a second fixture, <case>_amp, with the oracle's own
sensitivity: its samples after an early iteration n1, and the final samples
of a run whose state at n1 was moved by a relative 1e-12 (job_amp).

Usage:  python tests/golden/make_golden.py CASE [CASE ...]
Cases:  kerr_emri_6400x128, adjoint_3200x64_forward, batched_smallest4,
        adjoint_at_scale_first1000, and each of them with the suffix _amp
Writes tests/golden/<case>.npz (one file per case).
"""

import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import teuk_oracle as T  # noqa: E402
from paper_1001_3631_amd import workloads as W  # noqa: E402


def sample_rows(nth, extra=()):
    rows = {0, 1, 2, 3, 4, 7, 8, 15, 16, nth // 2 - 1, nth // 2, nth - 5, nth - 3, nth - 2, nth - 1}
    rows |= {int(j) for j in extra}
    return np.array(sorted(j for j in rows if 0 <= j < nth), dtype=np.int64)


def sample_cols(nr, i_ext, extra=()):
    cols = {0, 1, 2, 61, 62, 63, 123, 124, nr // 2, nr - 63, nr - 3, nr - 2, nr - 1, i_ext - 1, i_ext, i_ext + 1}
    cols |= {int(i) for i in extra}
    return np.array(sorted(i for i in cols if 0 <= i < nr), dtype=np.int64)


def sample_points(nth, nr, npts, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, nth, npts), rng.integers(0, nr, npts)


def pack(phi, pi, w, g, stride, extra_rows=(), extra_cols=(), npts=8192, seed=0, rect=None, full_rows=True):
    """Sample of the final state (phi, pi) and waveform w (see module doc)."""
    rows = sample_rows(g.nth, extra_rows) if full_rows else np.zeros(0, dtype=np.int64)
    cols = sample_cols(g.nr, g.i_ext, extra_cols)
    pj, pi_ = sample_points(g.nth, g.nr, npts, seed)
    out = dict(
        rows=rows, phi_rows=phi[rows], pi_rows=pi[rows],
        cols=cols, phi_cols=phi[:, cols], pi_cols=pi[:, cols],
        pts_j=pj, pts_i=pi_, phi_pts=phi[pj, pi_], pi_pts=pi[pj, pi_],
        row_norm_phi=np.sqrt(np.sum(np.abs(phi) ** 2, axis=1)),
        row_norm_pi=np.sqrt(np.sum(np.abs(pi) ** 2, axis=1)),
        norm_phi=np.sqrt(np.sum(np.abs(phi) ** 2)), norm_pi=np.sqrt(np.sum(np.abs(pi) ** 2)),
        max_phi=np.max(np.abs(phi)), max_pi=np.max(np.abs(pi)),
        wave_stride=np.int64(stride), wave=w[stride - 1::stride], wave_norm=np.sqrt(np.sum(np.abs(w) ** 2)),
        wave_max=np.max(np.abs(w)),
    )
    if rect is not None:
        j0, j1, i0, i1 = rect
        out.update(rect=np.array(rect, dtype=np.int64), phi_rect=phi[j0:j1, i0:i1], pi_rect=pi[j0:j1, i0:i1])
    return out


def circular_source(g, src, nsteps):
    orbit = T.circular_orbit(g.M, g.a, src["r0"], g.dt, nsteps)
    return T.Source(g, orbit, src["amplitude"], src["sigma_r_cells"], src["sigma_th_cells"], src["cutoff_sigmas"])


def source_cols(g, rs_p):
    i = int(np.rint((rs_p - g.rs_min) / g.hr))
    return (i - 40, i - 1, i, i + 1, i + 40)


# ---------------------------------------------------------------------------
# Workloads: each setup returns the oracle grid, initial state, source, the
# iteration count and the sampling (identical for every fixture of a case)
# ---------------------------------------------------------------------------

def setup_kerr_emri():
    cfg = W.KERR_EMRI
    g = T.Grid(**cfg["grid"])
    n = cfg["steps"]
    src = circular_source(g, cfg["source"], n)
    z = np.zeros((g.nth, g.nr), np.complex128)
    kw = dict(stride=100, extra_cols=source_cols(g, src.orbit["rs"][0]), seed=2)
    return g, z, z, src, n, kw, dict(workload=cfg["name"], steps=n, grid=cfg["grid"], source=cfg["source"],
                                     init="zero")


def setup_adjoint_forward():
    cfg = W.ADJOINT
    g = T.Grid(**cfg["grid"])
    n = cfg["steps"]
    src = circular_source(g, cfg["source"], n)
    phi0, pi0 = T.initial_pulse(g, **cfg["pulse"])
    kw = dict(stride=50, extra_cols=source_cols(g, src.orbit["rs"][0]), seed=4)
    return g, phi0, pi0, src, n, kw, dict(workload=cfg["name"], steps=n, grid=cfg["grid"], source=cfg["source"],
                                          pulse=cfg["pulse"])


BATCH_STEPS = 10000


def batched_smallest4():
    """The four smallest instances of the seed-3 batch: the first instance of
    the smallest grid level (1600 x 32) for each m in {1, 2, 3, 4}."""
    inst = W.batched_instances()
    pick = {}
    for k, d in enumerate(inst):
        if d["grid"]["nr"] == 1600 and d["grid"]["m"] not in pick:
            pick[d["grid"]["m"]] = k
    return [pick[m] for m in sorted(pick)]


def setup_batched(k):
    d0 = W.batched_instances()[k]
    g = T.Grid(**d0["grid"])
    phi0, pi0 = T.initial_pulse(g, **d0["pulse"])
    kw = dict(stride=50, npts=4096, seed=30 + k)
    return g, phi0, pi0, None, BATCH_STEPS, kw, dict(instance=k, grid=d0["grid"], pulse=d0["pulse"],
                                                     steps=BATCH_STEPS)


SCALE_STEPS = 1000
SCALE_PICK = (0, 7, 9, 13)   # spans a (0.04 .. 0.95), m (2, 3), e (0.12 .. 0.48), the closest orbit (p = 8.0)


def setup_scale(k):
    cfg = W.ADJOINT_AT_SCALE
    d0 = W.adjoint_at_scale_instances()[k]
    g = T.Grid(**d0["grid"])
    o = d0["orbit"]
    orbit = T.eccentric_orbit(g.M, g.a, o["p"], o["e"], o["chi0"], g.dt, SCALE_STEPS)
    s = cfg["source"]
    src = T.Source(g, orbit, s["amplitude"], s["sigma_r_cells"], s["sigma_th_cells"], s["cutoff_sigmas"])
    z = np.zeros((g.nth, g.nr), np.complex128)
    i_p = int(np.rint((orbit["rs"][-1] - g.rs_min) / g.hr))
    j_p = g.nth // 2
    rect = (j_p - 32, j_p + 33, i_p - 100, i_p + 101)
    kw = dict(stride=10, extra_cols=(i_p,), npts=4096, seed=50 + k, rect=rect, full_rows=False)
    return g, z, z, src, SCALE_STEPS, kw, dict(instance=k, grid=d0["grid"], orbit=o, source=s,
                                               steps=SCALE_STEPS, init="zero")


# ---------------------------------------------------------------------------
# Jobs
# ---------------------------------------------------------------------------

def job_main(setup, args, prefix):
    """The full run: samples of the final state and waveform."""
    g, p0, q0, src, n, kw, meta = setup(*args)
    phi, pi, w = T.evolve(g, p0, q0, n, src)
    return prefix, pack(phi, pi, w, g, **kw), meta


AMP_REL = 1e-12


def job_amp(setup, args, prefix, n1):
    """The oracle's own sensitivity.  Samples of the state after n1
    iterations (an early point where the GPU must still agree to 1e-12),
    and samples of the final state of a second run whose state at n1 was
    moved by a seeded random relative perturbation of 1e-12 (Phi and Pi each)
    and then evolved to the end.  The difference between these samples and
    the main fixture's is what a 1e-12 difference at n1 grows into by the
    end: the discrete problem's own amplification."""
    g, p0, q0, src, n, kw, meta = setup(*args)
    p, q, w1 = T.evolve(g, p0, q0, n1, src)
    mid = pack(p, q, w1, g, **dict(kw, stride=min(kw["stride"], n1)))
    rng = np.random.default_rng(12345)

    def perturb(x):
        d = rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)
        return x + AMP_REL * np.linalg.norm(x) / np.linalg.norm(d) * d

    p, q = perturb(p), perturb(q)
    w = [w1]
    for k in range(n1, n):
        p, q = T.step(g, p, q, k, src)
        w.append(p[:, g.i_ext].copy()[None, :])   # a copy: a view would keep every state alive
    end = pack(p, q, np.concatenate(w), g, **kw)
    d = {"mid_" + k: v for k, v in mid.items()}
    d.update({"pert_" + k: v for k, v in end.items()})
    d["n1"] = np.int64(n1)
    d["amp_rel"] = np.float64(AMP_REL)
    return prefix, d, dict(meta, n1=n1)


CASES = {
    "kerr_emri_6400x128": lambda: [(job_main, (setup_kerr_emri, (), ""))],
    "adjoint_3200x64_forward": lambda: [(job_main, (setup_adjoint_forward, (), ""))],
    "batched_smallest4": lambda: [(job_main, (setup_batched, (k,), f"i{k}_")) for k in batched_smallest4()],
    "adjoint_at_scale_first1000": lambda: [(job_main, (setup_scale, (k,), f"i{k}_")) for k in SCALE_PICK],
    "kerr_emri_6400x128_amp": lambda: [(job_amp, (setup_kerr_emri, (), "", 2000))],
    "adjoint_3200x64_forward_amp": lambda: [(job_amp, (setup_adjoint_forward, (), "", 2000))],
    "batched_smallest4_amp": lambda: [(job_amp, (setup_batched, (k,), f"i{k}_", 1000)) for k in batched_smallest4()],
    "adjoint_at_scale_first1000_amp": lambda: [(job_amp, (setup_scale, (k,), f"i{k}_", 250)) for k in SCALE_PICK],
}


def _run(fn_args):
    fn, args = fn_args
    t0 = time.time()
    out = fn(*args)
    return out, time.time() - t0


def make(case, jobs=4):
    todo = CASES[case]()
    arrays, meta = {}, []
    with ProcessPoolExecutor(max_workers=min(jobs, len(todo))) as ex:
        for (prefix, d, m), secs in ex.map(_run, todo):
            for k, v in d.items():
                arrays[prefix + k] = v
            m["oracle_seconds"] = round(secs, 1)
            meta.append(m)
            print(case, prefix or "-", f"{secs:.0f} s", flush=True)
    arrays["meta"] = np.array(json.dumps(dict(case=case, runs=meta,
                                              made_by="python tests/golden/make_golden.py " + case)))
    path = os.path.join(HERE, case + ".npz")
    np.savez_compressed(path, **arrays)
    print("wrote", path, os.path.getsize(path), "bytes", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for name in names:
        if name not in CASES:
            raise SystemExit(f"unknown case {name}; known: {', '.join(CASES)}")
    for name in names:
        make(name)
