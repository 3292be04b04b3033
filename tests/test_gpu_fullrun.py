"""Full-run GPU parity on the large workloads, against stored oracle results.

The fixtures under tests/golden/ are written by tests/golden/make_golden.py,
which runs only the CPU FP64 oracle (minutes to hours per workload, too long
for a test).  They hold samples of a state (whole theta rows, whole r*
columns, random points, the rectangle around a moving particle), the L2
norm of every theta row of the full state, and the waveform every stride-th
iteration.  The GPU runs the same workload in full through the C ABI and is
compared element by element on every stored sample.  Metrics:

* relative L2 over the samples of the joint solution vector u = (Phi, Pi),
  of Phi, of Pi, and of the waveform;
* the worst relative L2 of any stored row or column, so an error on the
  pole rows, a seam or the extraction column cannot hide in a global norm.
  A line's values come from neighbours at the field's scale, and after n
  iterations FP64 rounding has moved them by about sqrt(n) eps of that
  scale (the random-walk estimate of accumulated rounding), so a line
  whose norm is below sqrt(n) eps / 1e-12 of the largest line's cannot be
  resolved to a relative 1e-12 and is measured against that floor instead
  (near the theta = pi pole of the gradient workload Pi's rows are 1e-4 of
  the largest);
* the largest absolute difference over the samples against max|ref|;
* the L2 norm of every row of the full state against the oracle's (an error
  anywhere in a row moves its norm), relative to the global norm.

Two comparisons per workload:

* early, after n1 iterations: every metric <= 1e-12 (Pi's included);
* at the end of the full run: every metric <= max(1e-12, what the oracle's
  own sensitivity fixture shows), i.e. no larger than the difference that a
  relative 1e-12 perturbation of the oracle's state at n1 has grown into by
  the end.  Over tens of thousands of iterations these grids amplify any
  difference in rounding by many orders of magnitude (a mode at the light
  ring grows at a few hundredths per M; an outgoing s = -2 wave reflected
  by the outer Dirichlet wall is re-amplified about 1e4-fold as it falls
  in), so two correct FP64 evaluations of the same iteration cannot agree
  to 1e-12 at the end; the bound is derived from the oracle alone, with no
  chosen factor.
"""

import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1001_3631_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-12
EPS = np.finfo(np.float64).eps


def line_floor(n):
    """Smallest line norm, relative to the largest line's, resolvable to TOL
    after n iterations (see the module doc)."""
    return np.sqrt(n) * EPS / TOL


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1001_3631_amd import _lib
    _lib.load()


def load(name):
    path = os.path.join(GOLDEN, name + ".npz")
    if not os.path.exists(path):
        pytest.skip(f"fixture {name}.npz not generated (python tests/golden/make_golden.py {name})")
    z = np.load(path, allow_pickle=False)
    return {k: z[k] for k in z.files}


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def sub(fx, prefix):
    """Keys of fixture fx that start with prefix, prefix removed."""
    return {k[len(prefix):]: v for k, v in fx.items() if k.startswith(prefix)}


def sample_like(ref, phi, pi, w):
    """The GPU's full state (phi, pi) and waveform w sampled where ref was."""
    rows, cols = ref["rows"], ref["cols"]
    pj, pi_ = ref["pts_j"], ref["pts_i"]
    s = int(ref["wave_stride"])
    out = dict(phi_rows=phi[rows], pi_rows=pi[rows], phi_cols=phi[:, cols], pi_cols=pi[:, cols],
               phi_pts=phi[pj, pi_], pi_pts=pi[pj, pi_],
               row_norm_phi=np.sqrt(np.sum(np.abs(phi) ** 2, axis=1)),
               row_norm_pi=np.sqrt(np.sum(np.abs(pi) ** 2, axis=1)),
               wave=w[s - 1::s], wave_norm=np.sqrt(np.sum(np.abs(w) ** 2)))
    if "rect" in ref:
        j0, j1, i0, i1 = ref["rect"]
        out.update(phi_rect=phi[j0:j1, i0:i1], pi_rect=pi[j0:j1, i0:i1])
    return out


def _rel(d, ref):
    return float(np.sqrt(np.sum(np.abs(d) ** 2)) / max(np.sqrt(np.sum(np.abs(ref) ** 2)), 1e-300))


def metrics(a, ref, n):
    """Differences of sample set a (same keys as the fixture's) from ref,
    both after n iterations."""
    parts = ["rows", "cols", "pts"] + (["rect"] if "rect" in ref else [])
    gp = np.concatenate([a["phi_" + k].ravel() for k in parts])
    rp = np.concatenate([ref["phi_" + k].ravel() for k in parts])
    gq = np.concatenate([a["pi_" + k].ravel() for k in parts])
    rq = np.concatenate([ref["pi_" + k].ravel() for k in parts])
    assert np.max(np.abs(rp)) > 0, "empty reference sample"
    m = {"phi": _rel(gp - rp, rp), "pi": _rel(gq - rq, rq),
         "joint": float(np.sqrt((np.sum(np.abs(gp - rp) ** 2) + np.sum(np.abs(gq - rq) ** 2))
                                / (np.sum(np.abs(rp) ** 2) + np.sum(np.abs(rq) ** 2)))),
         "maxabs_phi": float(np.max(np.abs(gp - rp)) / ref["max_phi"]),
         "maxabs_pi": float(np.max(np.abs(gq - rq)) / max(float(ref["max_pi"]), 1e-300))}
    worst, where = 0.0, None
    for key, axis in (("rows", 1), ("cols", 0)):
        if ref["phi_" + key].size == 0:
            continue
        for f in ("phi_", "pi_"):
            g_, r_ = a[f + key], ref[f + key]
            dn = np.sqrt(np.sum(np.abs(g_ - r_) ** 2, axis=axis))
            rn = np.sqrt(np.sum(np.abs(r_) ** 2, axis=axis))
            top = max(float(np.max(rn)), 1e-300)
            e = dn / np.maximum(rn, line_floor(n) * top)
            k = int(np.argmax(e))
            if e[k] > worst:
                worst = float(e[k])
                where = (f + key, int(ref[key][k]), float(rn[k] / top), float(dn[k] / top))
    m["worst_line"] = worst
    if where is not None:
        print("  worst line (field, index, norm / largest, difference / largest):", where, flush=True)
    m["row_norms"] = float(max(np.max(np.abs(a["row_norm_phi"] - ref["row_norm_phi"])) / ref["norm_phi"],
                               np.max(np.abs(a["row_norm_pi"] - ref["row_norm_pi"])) / max(float(ref["norm_pi"]), 1e-300)))
    rw = ref["wave"]
    m["wave"] = _rel(a["wave"] - rw, rw) if np.max(np.abs(rw)) > 0 else float(np.max(np.abs(a["wave"])))
    m["wave_norm"] = abs(float(a["wave_norm"]) - float(ref["wave_norm"])) / max(float(ref["wave_norm"]), 1e-300)
    return m


def check(label, got, bound):
    print(label, {k: f"{v:.2e} <= {bound[k]:.2e}" for k, v in got.items()}, flush=True)
    bad = {k: (v, bound[k]) for k, v in got.items() if not v <= bound[k]}
    assert not bad, (label, bad)


def run_and_compare(label, main, amp, prefix, step, state):
    """step(n) advances the GPU run by n iterations and returns its waveform
    rows; state() returns the current (Phi, Pi) on the host.  Compares after
    n1 iterations and at the end (see the module doc)."""
    ref_end = sub(main, prefix)
    ref_mid = sub(amp, prefix + "mid_")
    pert = sub(amp, prefix + "pert_")
    n1 = int(amp[prefix + "n1"])
    n = int(json.loads(str(main["meta"]))["runs"][0]["steps"])
    w1 = host(step(n1))
    p, q = state()
    check(f"{label} after {n1} iterations", metrics(sample_like(ref_mid, p, q, w1), ref_mid, n1),
          {k: TOL for k in ("phi", "pi", "joint", "maxabs_phi", "maxabs_pi", "worst_line", "row_norms",
                            "wave", "wave_norm")})
    w2 = host(step(n - n1))
    p, q = state()
    w = np.concatenate([w1, w2])
    sens = metrics(pert, ref_end, n)   # what 1e-12 at n1 grows into, per metric
    check(f"{label} after {n} iterations", metrics(sample_like(ref_end, p, q, w), ref_end, n),
          {k: max(TOL, v / float(amp[prefix + "amp_rel"]) * TOL) for k, v in sens.items()})


def _circular(eng, grid, src, nsteps):
    orbit = eng.orbit_circular(src["r0"], 2 * nsteps + 1, M=grid["M"], a=grid["a"])
    eng.set_source(orbit, src["amplitude"], src["sigma_r_cells"], src["sigma_th_cells"], src["cutoff_sigmas"])


def _engine_run(eng):
    def state():
        p, q = eng.get_state()
        return host(p), host(q)
    return eng.step, state


def test_kerr_emri_6400x128_full_run_against_oracle():
    """Forced EMRI, 6400 x 128, 40000 iterations (every iteration's waveform
    at r* = 500M), in the launch configuration the benchmark uses."""
    from paper_1001_3631_amd.engine import Engine
    main, amp = load("kerr_emri_6400x128"), load("kerr_emri_6400x128_amp")
    cfg = W.KERR_EMRI
    eng = Engine(**cfg["grid"])
    eng.autotune()
    _circular(eng, cfg["grid"], cfg["source"], cfg["steps"])
    run_and_compare(f"kerr_emri_6400x128 {eng.tuning}", main, amp, "", *_engine_run(eng))
    eng.check_finite()


def test_adjoint_3200x64_forward_full_run_against_oracle():
    """The gradient workload's forward field: pulse plus circular source,
    3200 x 64, 20000 iterations, waveform at r* = 400M, in the launch
    configuration the benchmark uses."""
    from paper_1001_3631_amd.engine import Engine
    main, amp = load("adjoint_3200x64_forward"), load("adjoint_3200x64_forward_amp")
    cfg = W.ADJOINT
    eng = Engine(**cfg["grid"])
    eng.autotune()                        # the configuration the benchmark times
    eng.init_pulse(**cfg["pulse"])
    _circular(eng, cfg["grid"], cfg["source"], cfg["steps"])
    run_and_compare(f"adjoint_3200x64 forward {eng.tuning}", main, amp, "", *_engine_run(eng))


@pytest.mark.parametrize("mode", ["persistent", "per_iteration"])
def test_batched_smallest_instances_full_run_against_oracle(mode):
    """The four smallest instances of the 64-instance batch (1600 x 32, one
    per m), 10000 iterations, stepped together as one batch in each mode."""
    from paper_1001_3631_amd.engine import Batch
    main, amp = load("batched_smallest4"), load("batched_smallest4_amp")
    meta = json.loads(str(main["meta"]))
    ks = [r["instance"] for r in meta["runs"]]
    inst = W.batched_instances()
    b = Batch([inst[k]["grid"] for k in ks])
    b.set_mode(Batch.PERSISTENT if mode == "persistent" else Batch.PER_ITERATION)
    for e, k in zip(b.instances, ks):
        e.init_pulse(**inst[k]["pulse"])
    n1 = int(amp[f"i{ks[0]}_n1"])
    assert all(int(amp[f"i{k}_n1"]) == n1 for k in ks)
    n = meta["runs"][0]["steps"]
    w1 = b.step(n1)
    b.sync()
    w1 = [host(w) for w in w1]
    mids = [[host(x) for x in e.get_state()] for e in b.instances]
    w2 = b.step(n - n1)
    b.sync()
    for j, (e, k) in enumerate(zip(b.instances, ks)):
        ends = [host(x) for x in e.get_state()]
        calls = iter([w1[j], host(w2[j])])
        states = iter([mids[j], ends])
        run_and_compare(f"batched instance {k} ({mode})", sub_meta(main, k), amp, f"i{k}_",
                        lambda _n: torch.from_numpy(next(calls)), lambda: next(states))
    b.close()


def sub_meta(main, k):
    """main with the meta of instance k first (run_and_compare reads the
    iteration count from the first run)."""
    meta = json.loads(str(main["meta"]))
    runs = [r for r in meta["runs"] if r.get("instance") == k] + [r for r in meta["runs"] if r.get("instance") != k]
    out = dict(main)
    out["meta"] = np.array(json.dumps(dict(meta, runs=runs)))
    return out


def test_adjoint_at_scale_first_iterations_against_oracle():
    """Four of the 16 eccentric-orbit instances on 12800 x 256 (spanning a, m
    and e), their first 1000 iterations from zero data; each side builds its
    own orbit table from the geodesic equations."""
    from paper_1001_3631_amd.engine import Engine
    main, amp = load("adjoint_at_scale_first1000"), load("adjoint_at_scale_first1000_amp")
    meta = json.loads(str(main["meta"]))
    inst = W.adjoint_at_scale_instances()
    src = W.ADJOINT_AT_SCALE["source"]
    for run in meta["runs"]:
        k, n = run["instance"], run["steps"]
        d = inst[k]
        eng = Engine(**d["grid"])
        eng.autotune()                    # the configuration the benchmark times
        o = d["orbit"]
        orbit = eng.orbit_eccentric(o["p"], o["e"], 2 * n + 1, M=1.0, a=d["grid"]["a"], chi0=o["chi0"])
        eng.set_source(orbit, src["amplitude"], src["sigma_r_cells"], src["sigma_th_cells"], src["cutoff_sigmas"])
        run_and_compare(f"adjoint_at_scale instance {k} {eng.tuning}", sub_meta(main, k), amp, f"i{k}_",
                        *_engine_run(eng))
        eng.close()
