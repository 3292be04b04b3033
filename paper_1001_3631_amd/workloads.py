"""Synthetic workloads: instance descriptors and seeded input draws.

This module holds no arithmetic of the method (no coefficients, stepping,
orbits or sources): only grid sizes, physical parameters, and seeded random
draws (batch parameters, target noise, finite-difference directions).  Both
the oracle-based tests and the HIP path take their inputs from here.
"""

import numpy as np

# Common defaults: theta dissipation strength chosen by the stability analysis
# (the literal scheme is weakly unstable at the stiff pole rows).
KO_EPS = 0.5

SCHWARZSCHILD_PULSE = dict(  # 801 x 33, a = 0, 2000 steps, Gaussian pulse, no source
    name="schwarzschild_pulse_801x33",
    grid=dict(M=1.0, a=0.0, s=-2, m=2, nr=801, nth=33, rs_min=-100.0, rs_max=300.0, cfl=0.5,
              rs_extract=20.0, ko_eps=KO_EPS),
    steps=2000,
    pulse=dict(center=50.0, width=4.0, amplitude=1.0),
    source=None,
)

KERR_EMRI = dict(  # 6400 x 128, a = 0.9, circular orbit r0 = 10M, 40000 steps
    name="kerr_emri_6400x128",
    grid=dict(M=1.0, a=0.9, s=-2, m=2, nr=6400, nth=128, rs_min=-200.0, rs_max=600.0, cfl=0.5,
              rs_extract=500.0, ko_eps=KO_EPS),
    steps=40000,
    pulse=None,
    source=dict(r0=10.0, amplitude=1.0, sigma_r_cells=2.0, sigma_th_cells=2.0, cutoff_sigmas=8.0),
)

ADJOINT = dict(  # 3200 x 64, a = 0.7, 20000 steps, pulse + circular source, waveform misfit
    name="adjoint_3200x64",
    grid=dict(M=1.0, a=0.7, s=-2, m=2, nr=3200, nth=64, rs_min=-200.0, rs_max=600.0, cfl=0.5,
              rs_extract=400.0, ko_eps=KO_EPS),
    steps=20000,
    pulse=dict(center=50.0, width=4.0, amplitude=1.0),
    source=dict(r0=10.0, amplitude=1.0, sigma_r_cells=2.0, sigma_th_cells=2.0, cutoff_sigmas=8.0),
    target=dict(amplitude=1.25, center=52.0, noise_rel=0.01, seed=4),
    fd=dict(ndir=32, seed=44, h_rel=1e-3),
)

HBM_PLAIN = dict(  # forced EMRI physics on 25600 x 512: 420 MB per level, both levels 3.3x the 256 MB last-level cache
    name="kerr_emri_25600x512",
    grid=dict(M=1.0, a=0.9, s=-2, m=2, nr=25600, nth=512, rs_min=-200.0, rs_max=600.0, cfl=0.5,
              rs_extract=500.0, ko_eps=KO_EPS),
    steps=400,
    pulse=None,
    source=dict(r0=10.0, amplitude=1.0, sigma_r_cells=2.0, sigma_th_cells=2.0, cutoff_sigmas=8.0),
)

SCALE_GRID = dict(  # the 12800 x 256 grid of the 16-instance workload: 105 MB per level, inside the last-level cache
    name="kerr_emri_12800x256",
    grid=dict(M=1.0, a=0.9, s=-2, m=2, nr=12800, nth=256, rs_min=-200.0, rs_max=600.0, cfl=0.5,
              rs_extract=500.0, ko_eps=KO_EPS),
    steps=2000,
    pulse=None,
    source=dict(r0=10.0, amplitude=1.0, sigma_r_cells=2.0, sigma_th_cells=2.0, cutoff_sigmas=8.0),
)


ALL_M = dict(  # every m of one circular orbit on the EMRI grid, stepped as one batch
    name="all_m_6400x128",
    # cfl 0.25: the m = 3, 4 modes need it (as in the batched instances below)
    grids=[dict(KERR_EMRI["grid"], m=m, cfl=0.25) for m in (1, 2, 3, 4)],
    steps=4000,
    source=dict(KERR_EMRI["source"]),
)


def batched_instances(seed=3, n=64):
    """64 independent evolutions: m uniform in {1,2,3,4}, a uniform in [0, 0.99],
    grid level uniform in {0..3} (1600*2^l x 32*2^l), pulse centre uniform in
    [20, 80] M.  cfl 0.25: at cfl 0.5 the m = 3, 4 modes at small a put the
    stiff pole mode beyond what the dissipation can hold."""
    rng = np.random.default_rng(seed)
    m = rng.integers(1, 5, n)
    a = rng.uniform(0.0, 0.99, n)
    lvl = rng.integers(0, 4, n)
    c = rng.uniform(20.0, 80.0, n)
    out = []
    for k in range(n):
        out.append(dict(
            grid=dict(M=1.0, a=float(a[k]), s=-2, m=int(m[k]), nr=int(1600 * 2 ** lvl[k]),
                      nth=int(32 * 2 ** lvl[k]), rs_min=-200.0, rs_max=600.0, cfl=0.25,
                      rs_extract=100.0, ko_eps=KO_EPS),
            pulse=dict(center=float(c[k]), width=4.0, amplitude=1.0)))
    return out


ADJOINT_AT_SCALE = dict(  # 16 eccentric-orbit instances on 12800 x 256, forward + checkpointed adjoint
    name="adjoint_at_scale_16x12800x256",
    instances=16,
    seed=5,
    steps=50000,
    source=dict(amplitude=1.0, sigma_r_cells=2.0, sigma_th_cells=2.0, cutoff_sigmas=8.0),
    # target: the same instance's waveform at source amplitude 0.9 (zero
    # initial data, so w is linear in A and the target is 0.9 w)
    target_amplitude=0.9,
)


def adjoint_at_scale_instances(seed=5, n=16):
    """16 instances on 12800 x 256: a uniform in [0, 0.95], m uniform in
    {2, 3}, eccentric equatorial orbits with p uniform in [8, 14] M, e
    uniform in [0, 0.5] and anomaly at t = 0 uniform in [0, 2 pi).  cfl 0.25
    (as for the other batches with m = 3); extraction at r* = 100M, which the
    signal from the orbit reaches well within the run (at 50000 iterations
    the runs span 200-310 M)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 0.95, n)
    m = rng.integers(2, 4, n)
    p = rng.uniform(8.0, 14.0, n)
    e = rng.uniform(0.0, 0.5, n)
    chi0 = rng.uniform(0.0, 2.0 * np.pi, n)
    out = []
    for k in range(n):
        out.append(dict(
            grid=dict(M=1.0, a=float(a[k]), s=-2, m=int(m[k]), nr=12800, nth=256, rs_min=-200.0,
                      rs_max=600.0, cfl=0.25, rs_extract=100.0, ko_eps=KO_EPS),
            orbit=dict(p=float(p[k]), e=float(e[k]), chi0=float(chi0[k]))))
    return out


def complex_normal(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def target_noise(shape, scale, seed=4):
    """Complex N(0, scale^2) noise for the target waveform."""
    rng = np.random.default_rng(seed)
    return scale * complex_normal(rng, shape) / np.sqrt(2.0)


def fd_directions(nth, nr, ndir=32, seed=44):
    """Unit directions over (Re, Im of Phi0, Pi0; A) for finite differences."""
    rng = np.random.default_rng(seed)
    dirs = []
    for _ in range(ndir):
        vp = complex_normal(rng, (nth, nr))
        vq = complex_normal(rng, (nth, nr))
        vA = rng.standard_normal()
        nrm = np.sqrt(np.sum(np.abs(vp) ** 2) + np.sum(np.abs(vq) ** 2) + vA ** 2)
        dirs.append((vp / nrm, vq / nrm, vA / nrm))
    return dirs


def random_state(nth, nr, seed):
    rng = np.random.default_rng(seed)
    return complex_normal(rng, (nth, nr)), complex_normal(rng, (nth, nr))


def synthetic_waveforms(ms, nsteps, nth, dt, seed=6):
    """Seeded smooth stand-ins for extracted waveforms of several m modes,
    (nsteps + 1, nth) complex each: a few damped oscillations in t with
    random amplitudes, frequencies and angular profiles (low powers of sin
    and cos of theta_j = j pi/(nth - 1))."""
    rng = np.random.default_rng(seed)
    th = np.arange(nth) * np.pi / (nth - 1)
    t = np.arange(nsteps + 1) * dt
    out = []
    for _ in ms:
        w = np.zeros((nsteps + 1, nth), dtype=np.complex128)
        for _ in range(3):
            prof = sum(complex_normal(rng, ()) * np.sin(th) ** k * np.cos(th) ** l for k in range(3) for l in range(2))
            om = rng.uniform(0.05, 0.6)
            ga = rng.uniform(0.0, 0.02)
            w += np.exp((-1j * om - ga) * t)[:, None] * prof[None, :]
        out.append(w)
    return out
