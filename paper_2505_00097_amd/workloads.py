"""Seeded synthetic inputs (no method arithmetic here).

Holds the workload definitions (grid sizes, punctures, step counts), the
seeded draws of ensemble and served jobs, and smooth random states used to
exercise every term of the right-hand sides. Both the HIP path's tests and
the oracle side take their inputs from here.
"""
import numpy as np

SINH_SPHERICAL, SINH_CYLINDRICAL, SPHERICAL = 0, 1, 2

# Workloads: synthetic stand-ins for the paper's runs (Brill-Lindquist data
# instead of TwoPunctures, which is an external spectral solver).
WORKLOADS = {
    "tiny_sinhspherical_32x16x2": dict(
        coord=SINH_SPHERICAL, N=(32, 16, 2), ampl=(10.0,) * 3, sinhw=(0.2,) * 3, cfl=0.5,
        masses=[1.0], positions=[(0.0, 0.0, 0.0)], steps=10, eta=2.0),
    "headon_sinhcylindrical_128x2x256": dict(
        coord=SINH_CYLINDRICAL, N=(128, 2, 256), ampl=(20.0,) * 3, sinhw=(0.2,) * 3, cfl=0.5,
        masses=[0.5, 0.5], positions=[(0.0, 0.0, 0.5), (0.0, 0.0, -0.5)], steps=1000, eta=2.0,
        h_every=50),
    "vacuum3d_sinhspherical_256x128x64": dict(
        coord=SINH_SPHERICAL, N=(256, 128, 64), ampl=(10.0,) * 3, sinhw=(0.2,) * 3, cfl=0.5,
        masses=[0.6, 0.4], positions=[(0.7, 0.0, 0.0), (-0.7, 0.0, 0.0)], steps=200, eta=2.0),
    # the paper's single-node benchmark grid (plain spherical, r_max = 7.5)
    "paper_single_node_spherical_72x12x24": dict(
        coord=SPHERICAL, N=(72, 12, 24), ampl=(7.5,) * 3, sinhw=(0.2,) * 3, cfl=0.5,
        masses=[0.5, 0.5], positions=[(0.0, 0.0, 0.5), (0.0, 0.0, -0.5)], steps=8428, eta=2.0),
}


def headon_job(q, d, n_rho, ampl=20.0, sinhw=0.2):
    """Head-on BL job: m1 = q/(1+q) at z = +d/2, m2 = 1/(1+q) at z = -d/2 on a
    SinhCylindrical grid N = (n_rho, 2, 2 n_rho)."""
    return dict(coord=SINH_CYLINDRICAL, N=(int(n_rho), 2, 2 * int(n_rho)), ampl=(ampl,) * 3,
                sinhw=(sinhw,) * 3, cfl=0.5, masses=[q / (1.0 + q), 1.0 / (1.0 + q)],
                positions=[(0.0, 0.0, d / 2.0), (0.0, 0.0, -d / 2.0)], eta=2.0)


def batched_jobs(n=64, seed=250500097):
    """Ensemble: per job q ~ U[1,4], d ~ U[0.8,2.0], N_rho ~ U{48..192}."""
    rng = np.random.default_rng(seed)
    jobs = []
    for _ in range(n):
        q = rng.uniform(1.0, 4.0)
        d = rng.uniform(0.8, 2.0)
        nr = int(rng.integers(48, 193))
        jobs.append(headon_job(q, d, nr))
    return jobs


def served_jobs(n=256, seed=250500098, rate=4.0):
    """Poisson arrivals (rate jobs/s): q ~ U[1,8], d ~ U[0.8,3.0],
    N_rho in {64,96,128,192}, steps ~ U{200..2000}."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for _ in range(n):
        t += rng.exponential(1.0 / rate)
        q = rng.uniform(1.0, 8.0)
        d = rng.uniform(0.8, 3.0)
        nr = int(rng.choice([64, 96, 128, 192]))
        steps = int(rng.integers(200, 2001))
        job = headon_job(q, d, nr)
        job.update(arrival=t, steps=steps)
        jobs.append(job)
    return jobs


def smooth_random_state(n_total, seed, shift_amp=0.3):
    """A smooth random state of shape (24, n2, n1, n0), built from a few low
    Fourier modes of the grid indices: h_ij, a_ij, lambda, B, K of size 0.1-0.3,
    W and alpha in [0.4, 1], and a shift that takes both signs."""
    n0, n1, n2 = n_total
    rng = np.random.default_rng(seed)
    I2, I1, I0 = np.meshgrid(np.arange(n2) / n2, np.arange(n1) / n1, np.arange(n0) / n0, indexing="ij")

    def field(amp, offset=0.0, modes=3):
        f = np.full(I0.shape, offset)
        for _ in range(modes):
            k = rng.integers(0, 3, 3)
            ph = rng.uniform(0, 2 * np.pi)
            f += amp / modes * rng.uniform(0.5, 1.0) * np.sin(2 * np.pi * (k[0] * I0 + k[1] * I1 + k[2] * I2) + ph)
        return f

    y = np.zeros((24, n2, n1, n0))
    for g in range(6):
        y[g] = field(0.3)                   # aDD
        y[11 + g] = field(0.1)              # hDD
    y[6] = field(0.25, 0.7)                 # alpha
    y[10] = field(0.25, 0.7)                # cf
    for i in range(3):
        y[7 + i] = field(0.2)               # betU
        y[17 + i] = field(0.2)              # lambdaU
        y[21 + i] = field(shift_amp)        # vetU
    y[20] = field(0.3)                      # trK
    return y
