"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module only draws and lays out inputs (mesh sizes, conductivity fields,
stimulus weights, random cell states, method parameters); it holds none of the
method's arithmetic.  Every random quantity comes from numpy.random.default_rng
with an explicit seed.

Workloads (the tissue slabs of the benchmark; the paper's own runs use a
spiral-wave initial state on [0, 100 mm]^d, replaced here by the TTP06 rest
state plus a stimulus):
  cable1d   1D cable, 128 nodes, dx 0.01 cm, 3-point Laplacian, sigma 1 mS/cm,
            stimulus 50 uA/cm^2 for 1 ms on nodes 0-4; M 4, K 4, dt 0.05, T 10.
  slab2d    2D 512 x 512, dx 0.025 cm, 5-point, sigma 1; stimulus on the corner
            16 x 16 square, 50 uA/cm^2 for 1 ms; M 6, K 6, dt 0.05, T 20;
            CG to 1e-12 relative residual.
  slab3d    3D 192 x 96 x 48, dx 0.025 cm, 7-point, sigma (3, 1, 1) with the
            fibre along x; stimulus on the face x in {node 0, 1}; two-level PFASST,
            P 16, fine M 6, coarse M 3 on the mesh coarsened 2x; dt 0.1, T 32.
  batch2d   64 tissues with side lengths uniform in 64..512, per-node sigma
            exp(0.3 N(0,1)) mS/cm, one random 8 x 8 stimulus patch per tissue;
            M 4, K 4, dt 0.05, T 10.
Common: chi 1400 /cm, Cm 1 uF/cm^2, TTP06 epicardial rest state.
"""
import numpy as np

CHI = 1400.0
CM = 1.0
STIM_AMP = 50.0
STIM_T0 = 0.0
STIM_DUR = 1.0

# physiological ranges used to draw random TTP06 states (field order of the model)
STATE_RANGES = (
    (-90.0, 40.0),        # V
    (5e-5, 1.5e-3),       # Ca_i
    (0.5, 4.5),           # Ca_SR
    (1e-4, 2e-2),         # Ca_ss
    (7.0, 12.0),          # Na_i
    (130.0, 140.0),       # K_i
    (0.5, 1.0),           # Rbar
) + ((0.0, 1.0),) * 12    # gates


def random_states(n, seed=0):
    """n random cell states (19, n) inside physiological ranges, plus the
    special voltages 15 mV and -40 mV (the removable singularity of I_CaL and
    the branch point of the h, j gates) on the first two nodes."""
    rng = np.random.default_rng(seed)
    y = np.empty((len(STATE_RANGES), n))
    for f, (lo, hi) in enumerate(STATE_RANGES):
        y[f] = rng.uniform(lo, hi, n)
    if n >= 2:
        y[0, 0] = 15.0
        y[0, 1] = -40.0
    return y


def corner_weights(dims, size):
    """Stimulus weight 1 on the corner box [0, size)^d, 0 elsewhere (x fastest)."""
    nx, ny, nz = (tuple(dims) + (1, 1, 1))[:3]
    w = np.zeros((nz, ny, nx))
    sx, sy, sz = (tuple(size) + (1, 1, 1))[:3]
    w[:sz, :sy, :sx] = 1.0
    return w.ravel()


def face_weights(dims, depth):
    """Stimulus weight 1 on the nodes with x index < depth (a planar face)."""
    nx, ny, nz = (tuple(dims) + (1, 1, 1))[:3]
    w = np.zeros((nz, ny, nx))
    w[:, :, :depth] = 1.0
    return w.ravel()


def workload(name, dims=None, t_end=None):
    """Problem and method parameters of a named workload.  dims and t_end
    override the sizes (for reduced parity cases)."""
    if name == "cable1d":
        d = tuple(dims) if dims else (128,)
        return dict(name=name, dims=d, dx=0.01, sigma=(1.0, 1.0, 1.0), sigma_node=None,
                    chi=CHI, Cm=CM, stim_w=corner_weights(d, (5,)), stim_amp=STIM_AMP,
                    stim_t0=STIM_T0, stim_dur=STIM_DUR, M=4, K=4, dt=0.05,
                    t_end=t_end or 10.0, cg_rtol=1e-12)
    if name == "slab2d":
        d = tuple(dims) if dims else (512, 512)
        s = min(16, d[0], d[1])
        return dict(name=name, dims=d, dx=0.025, sigma=(1.0, 1.0, 1.0), sigma_node=None,
                    chi=CHI, Cm=CM, stim_w=corner_weights(d, (s, s)), stim_amp=STIM_AMP,
                    stim_t0=STIM_T0, stim_dur=STIM_DUR, M=6, K=6, dt=0.05,
                    t_end=t_end or 20.0, cg_rtol=1e-12)
    if name == "slab3d":
        d = tuple(dims) if dims else (192, 96, 48)
        return dict(name=name, dims=d, dx=0.025, sigma=(3.0, 1.0, 1.0), sigma_node=None,
                    chi=CHI, Cm=CM, stim_w=face_weights(d, 2), stim_amp=STIM_AMP,
                    stim_t0=STIM_T0, stim_dur=STIM_DUR, M=6, Mc=3, P=16, dt=0.1,
                    t_end=t_end or 32.0, cg_rtol=1e-12, space_coarsen=2)
    raise KeyError(name)


def batch2d_tissues(n_tissues=64, seed=0, lo=64, hi=512):
    """The ragged batch: per tissue (nx, ny), per-node sigma field and an 8 x 8
    stimulus patch at a uniform random in-bounds corner."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_tissues):
        nx = int(rng.integers(lo, hi + 1))
        ny = int(rng.integers(lo, hi + 1))
        sig = 1.0 * np.exp(0.3 * rng.standard_normal(nx * ny))
        px = int(rng.integers(0, nx - 8 + 1))
        py = int(rng.integers(0, ny - 8 + 1))
        w = np.zeros((ny, nx))
        w[py:py + 8, px:px + 8] = 1.0
        out.append(dict(name="batch2d", dims=(nx, ny), dx=0.025, sigma=(1.0, 1.0, 1.0),
                        sigma_node=sig, chi=CHI, Cm=CM, stim_w=w.ravel(), stim_amp=STIM_AMP,
                        stim_t0=STIM_T0, stim_dur=STIM_DUR, M=4, K=4, dt=0.05, t_end=10.0,
                        cg_rtol=1e-12))
    return out
