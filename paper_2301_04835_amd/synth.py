"""Seeded synthetic inputs shaped like the paper's benchmark workloads.

This module holds no arithmetic of the biasing method: it only draws
positions, hill centres and heights, system forces and walker sizes from
NumPy's seeded generators, so that the HIP path and the CPU oracle can be
fed identical values.  Stored dtypes are what the engine would hand over
(float32 unless a workload asks for float64).

Workloads (the paper's own systems are not available, so each is a stand-in
with the shape of the paper's case):
  * a 22-atom backbone-like chain with two dihedral CVs sharing three atoms,
    the shape of the alanine-dipeptide phi/psi example of the appendix;
  * a 50,000-atom box with a radius-of-gyration and a coordination-number CV;
  * batches of walkers of uneven sizes (replicas, Sec. 2 on parallel runs).
"""
import numpy as np

TWO_PI = 2.0 * np.pi


def rng(seed):
    return np.random.default_rng(seed)


def chain_template(n_atoms, seed, bond=0.15, angle_deg=110.0):
    """Unbranched chain with fixed bond length and bond angle and random
    torsions, placed atom by atom (natural-extension reference frame)."""
    g = rng(seed)
    th = np.deg2rad(angle_deg)
    x = np.zeros((n_atoms, 3))
    if n_atoms > 1:
        x[1] = [bond, 0.0, 0.0]
    if n_atoms > 2:
        x[2] = x[1] + bond * np.array([-np.cos(th), np.sin(th), 0.0])
    for i in range(3, n_atoms):
        tor = g.uniform(-np.pi, np.pi)
        a, b, c = x[i - 3], x[i - 2], x[i - 1]
        bc = c - b
        bc /= np.linalg.norm(bc)
        n = np.cross(b - a, bc)
        n /= np.linalg.norm(n)
        m = np.cross(n, bc)
        d2 = np.array([-bond * np.cos(th), bond * np.sin(th) * np.cos(tor), bond * np.sin(th) * np.sin(tor)])
        x[i] = c + d2[0] * bc + d2[1] * m + d2[2] * n
    return x


def backbone_cvs(first=4):
    """Two dihedrals sharing three atoms: phi = (f, f+1, f+2, f+3),
    psi = (f+1, f+2, f+3, f+4)."""
    return [
        {"kind": "dihedral", "idx": [first, first + 1, first + 2, first + 3]},
        {"kind": "dihedral", "idx": [first + 1, first + 2, first + 3, first + 4]},
    ]


def noisy_frames(template, n_frames, seed, sd=0.02, dtype=np.float64):
    """Frames = template + N(0, sd^2) per coordinate (nm)."""
    g = rng(seed)
    t = np.asarray(template, dtype=np.float64)
    return (t[None] + g.normal(0.0, sd, size=(n_frames,) + t.shape)).astype(dtype)


def uniform_centers(K, D, seed, lo=-np.pi, hi=np.pi):
    """Hill centres uniform in [lo, hi)^D, stored as float32 (K x D)."""
    return rng(seed).uniform(lo, hi, size=(K, D)).astype(np.float32)


def uniform_heights(K, seed, lo=0.5, hi=1.5):
    """Hill heights uniform in [lo, hi) kJ/mol, stored as float32."""
    return rng(seed).uniform(lo, hi, size=K).astype(np.float32)


# ------------------------------------------------------------------------- #
# 22-atom WTMD workload: phi/psi of a backbone-like chain, 2,000 hills,     #
# sigma 0.35 rad, w 1.2 kJ/mol, bias factor 6, T 300 K, stride 500.         #
# ------------------------------------------------------------------------- #
WTMD22 = dict(n_atoms=22, n_hills=2000, sigma=(0.35, 0.35), w=1.2, bias_factor=6.0, T=300.0, stride=500,
              n_steps=1000, noise=0.02)


def wtmd22_inputs(n_steps=None, seed=1):
    p = WTMD22
    n_steps = p["n_steps"] if n_steps is None else n_steps
    tmpl = chain_template(p["n_atoms"], seed)
    frames = noisy_frames(tmpl, n_steps, seed + 100, p["noise"], np.float64)
    centers = uniform_centers(p["n_hills"], 2, seed + 200)
    return {"template": tmpl, "frames": frames, "centers": centers, "cvs": backbone_cvs(4)}


# ------------------------------------------------------------------------- #
# 50,000-atom ABF workload: Rg of atoms [0, 500), coordination number       #
# between A = [500, 1500) and B = [1500, 2500) (r0 0.5 nm, n 6, m 12),       #
# uniform positions in a 10 nm cube, 100 x 100 grid.                         #
# ------------------------------------------------------------------------- #
# grid range: mean +- ~5 sd of (Rg, CN) over a seeded 300-frame pilot
# (Rg 4.996 +- 0.059 nm, CN 820.8 +- 19.5), rounded outwards
ABF50K = dict(n_atoms=50000, box=10.0, n_rg=500, n_a=1000, n_b=1000, r0=0.5, n=6, m=12, nbins=(100, 100),
              lo=(4.7, 720.0), hi=(5.3, 920.0), n_threshold=500, n_steps=10000, fsys_sd=100.0)


def abf50k_cvs(overlap=False):
    p = ABF50K
    rg = list(range(0, p["n_rg"]))
    a0 = p["n_rg"]
    a = list(range(a0, a0 + p["n_a"]))
    b0 = a0 + p["n_a"] - (p["n_a"] // 2 if overlap else 0)
    b = list(range(b0, b0 + p["n_b"]))
    return [
        {"kind": "gyration", "idx": rg},
        {"kind": "coordination", "a": a, "b": b, "r0": p["r0"], "n": p["n"], "m": p["m"], "rcut": 0.0,
         "normalize": False},
    ]


def abf50k_box(seed=2, n_atoms=None):
    p = ABF50K
    n = p["n_atoms"] if n_atoms is None else n_atoms
    return rng(seed).uniform(0.0, p["box"], size=(n, 3)).astype(np.float32)


def abf50k_frames(n_steps, seed=2, n_active=2500):
    """Per step: fresh uniform positions of the active atoms and system
    forces ~ N(0, fsys_sd^2) kJ/mol/nm on them (float32)."""
    p = ABF50K
    g = rng(seed + 1000)
    pos = g.uniform(0.0, p["box"], size=(n_steps, n_active, 3)).astype(np.float32)
    f = g.normal(0.0, p["fsys_sd"], size=(n_steps, n_active, 3)).astype(np.float32)
    return pos, f


# ------------------------------------------------------------------------- #
# Batched walkers: 256 walkers, atoms log-uniform in [22, 5000], private    #
# hill counts uniform in [1k, 50k], two dihedrals on each walker's first    #
# atoms, hill centres uniform on the torus, heights U[0.5, 1.5] kJ/mol.     #
# ------------------------------------------------------------------------- #
WALKERS256 = dict(n_walkers=256, atoms_lo=22, atoms_hi=5000, hills_lo=1000, hills_hi=50000, sigma=(0.35, 0.35),
                  w=1.2, bias_factor=6.0, T=300.0, stride=500)


def walker_sizes(n_walkers, seed, atoms_lo=22, atoms_hi=5000, hills_lo=1000, hills_hi=50000):
    g = rng(seed)
    n_atoms = np.rint(np.exp(g.uniform(np.log(atoms_lo), np.log(atoms_hi), size=n_walkers))).astype(np.int64)
    n_hills = g.integers(hills_lo, hills_hi + 1, size=n_walkers).astype(np.int64)
    return n_atoms, n_hills


def walkers_inputs(n_walkers=256, seed=3, atoms=(22, 5000), hills=(1000, 50000), dtype=np.float32):
    """Positions of all walkers concatenated (sum n_w x 3), atom offsets,
    hill counts, hill centres and heights of all walkers concatenated."""
    n_atoms, n_hills = walker_sizes(n_walkers, seed, atoms[0], atoms[1], hills[0], hills[1])
    g = rng(seed + 1)
    tmpl = chain_template(8, seed + 2)
    atom_off = np.concatenate([[0], np.cumsum(n_atoms)]).astype(np.int64)
    pos = g.uniform(-1.0, 1.0, size=(int(atom_off[-1]), 3))
    for w in range(n_walkers):
        o = atom_off[w]
        # first atoms of every walker: the chain template, jittered and shifted
        pos[o:o + 8] = tmpl + g.normal(0.0, 0.02, size=tmpl.shape) + g.uniform(-1, 1, size=3)
    K = int(n_hills.sum())
    centers = g.uniform(-np.pi, np.pi, size=(K, 2)).astype(np.float32)
    heights = g.uniform(0.5, 1.5, size=K).astype(np.float32)
    hill_off = np.concatenate([[0], np.cumsum(n_hills)]).astype(np.int64)
    return {"pos": pos.astype(dtype), "atom_off": atom_off, "n_atoms": n_atoms, "n_hills": n_hills,
            "hill_off": hill_off, "centers": centers, "heights": heights, "cvs": backbone_cvs(1)}


def chain_walkers(n_walkers, n_atoms=22, seed=4, dtype=np.float32):
    """n_walkers independent chains of n_atoms atoms (each its own random
    torsions, so the walkers' dihedrals spread over the torus), stacked:
    positions (n_walkers * n_atoms, 3) and walker atom offsets."""
    pos = np.concatenate([chain_template(n_atoms, seed * 100003 + w) for w in range(n_walkers)])
    return pos.astype(dtype), np.arange(n_walkers + 1, dtype=np.int64) * n_atoms


# ------------------------------------------------------------------------- #
# Three coordination numbers over 20,000-atom groups: per walker 60,000      #
# atoms uniform in a 12 nm periodic box, groups A, B, C = consecutive thirds, #
# CN_AB, CN_BC, CN_CA (r0 0.5 nm, n 6, m 12, hard cut 1.2 nm, divided by     #
# |A|), one shared list of 10^6 hills of width 0.2 around the expected CN.   #
# ------------------------------------------------------------------------- #
CN3 = {"n_group": 20000, "box": 12.0, "r0": 0.5, "rcut": 1.2, "sigma": 0.2,
       # expected per-atom CN at density 20000 / 12^3 nm^-3 (the integral of
       # 4 pi r^2 rho s(r) to the cut), the centre of the hill cloud
       "cn_mean": 9.0817, "hill_sd": 0.3}


def cn3_cvs(n_group=20000, r0=0.5, rcut=1.2):
    g = [list(range(k * n_group, (k + 1) * n_group)) for k in range(3)]
    mk = lambda a, b: {"kind": "coordination", "a": a, "b": b, "r0": r0, "n": 6, "m": 12, "rcut": rcut,
                       "normalize": True}
    return [mk(g[0], g[1]), mk(g[1], g[2]), mk(g[2], g[0])]


def cn3_positions(n_walkers, n_group=20000, box=12.0, seed=5):
    """(n_walkers * 3 n_group, 3) float32 positions uniform in [0, box)^3 and
    the walker atom offsets."""
    n = 3 * n_group
    pos = rng(seed).uniform(0.0, box, size=(n_walkers * n, 3)).astype(np.float32)
    return pos, np.arange(n_walkers + 1, dtype=np.int64) * n


def cn3_hills(K, seed=6, mean=9.0817, sd=0.3):
    """K hill centres N(mean, sd^2) in each of the three CVs (float32, K x 3)
    and heights U[0.5, 1.5] kJ/mol."""
    g = rng(seed)
    return (mean + sd * g.normal(size=(K, 3))).astype(np.float32), g.uniform(0.5, 1.5, size=K).astype(np.float32)
