"""ctypes binding of the FP64 C oracle (``oracle.c``); test infrastructure only.

The shared object is built with gcc next to the source by ``build()`` (the
package build calls it every time); ``lib()`` rebuilds it only when it is
missing or was built from other source text (a sha256 of ``oracle.c`` is
kept beside it), so copying the tree, which may reorder file times, never
starts a compiler in a process that only checks results.  No fast-math:
``-O2 -fno-fast-math``.
"""
import ctypes
import hashlib
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_STAMP = _LIB + ".src-sha256"

KB = 0.008314462618  # kJ/(mol K): R/1000, CODATA 2018 (exact)


def _src_sha():
    with open(_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _built_from_current_source():
    if not (os.path.exists(_LIB) and os.path.exists(_STAMP)):
        return False
    with open(_STAMP) as f:
        return f.read().strip() == _src_sha()


def build(force=False):
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc, OpenMP, no fast-math)."""
    if not force and _built_from_current_source():
        return _LIB
    sha = _src_sha()
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fno-fast-math", "-fPIC", "-shared", "-fopenmp", "-std=c11",
           _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    with open(_STAMP + ".tmp%d" % os.getpid(), "w") as f:
        f.write(sha + "\n")
    os.replace(_STAMP + ".tmp%d" % os.getpid(), _STAMP)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.orc_dihedral.argtypes = [P, P, P]
        L.orc_dihedral.restype = ctypes.c_int
        L.orc_gyration.argtypes = [P, i64, P, P]
        L.orc_gyration.restype = ctypes.c_int
        L.orc_switch.argtypes = [f64, f64, ctypes.c_int, ctypes.c_int, P, P]
        L.orc_switch.restype = None
        L.orc_coordination.argtypes = [P, i64, P, i64, P, i64, f64, ctypes.c_int, ctypes.c_int, f64, P,
                                       ctypes.c_int, P, P]
        L.orc_coordination.restype = ctypes.c_int
        L.orc_hillsum.argtypes = [ctypes.c_int, P, i64, P, P, P, P, P, P]
        L.orc_hillsum.restype = None
        L.orc_hillsum_batch.argtypes = [ctypes.c_int, ctypes.c_int, P, P, i64, P, P, P, P, P, P, ctypes.c_int]
        L.orc_hillsum_batch.restype = None
        L.orc_wt_height.argtypes = [f64, f64, f64]
        L.orc_wt_height.restype = f64
        L.orc_wt_sequence.argtypes = [ctypes.c_int, i64, P, f64, f64, P, P, ctypes.c_int, P]
        L.orc_wt_sequence.restype = None
        _ = (i32,)
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def dihedral(r):
    """O1: dihedral angle of four points r (4x3) and dphi/dr (4x3)."""
    r = _f64(r).reshape(4, 3)
    phi = np.zeros(1)
    g = np.zeros((4, 3))
    rc = lib().orc_dihedral(_p(r), _p(phi), _p(g))
    if rc != 0:
        raise ValueError("dihedral undefined for collinear points")
    return float(phi[0]), g


def gyration(pos):
    """O2: unweighted radius of gyration of pos (n x 3) and dRg/dr."""
    pos = _f64(pos).reshape(-1, 3)
    rg = np.zeros(1)
    g = np.zeros_like(pos)
    rc = lib().orc_gyration(_p(pos), pos.shape[0], _p(rg), _p(g))
    if rc != 0:
        raise ValueError("radius of gyration undefined")
    return float(rg[0]), g


def switch(r, r0, n, m):
    """O3: rational switching function s(r) and ds/dr."""
    s = np.zeros(1)
    ds = np.zeros(1)
    lib().orc_switch(float(r), float(r0), int(n), int(m), _p(s), _p(ds))
    return float(s[0]), float(ds[0])


def coordination(pos, a, b, r0, n, m, rcut=0.0, box=None, normalize=False):
    """O3: coordination number between index groups a and b, and dCN/dr for
    every atom of pos (natoms x 3).  box: orthorhombic edge lengths or None."""
    pos = _f64(pos).reshape(-1, 3)
    a = np.ascontiguousarray(a, dtype=np.int32)
    b = np.ascontiguousarray(b, dtype=np.int32)
    L = None if box is None else _f64(box).reshape(3)
    cn = np.zeros(1)
    g = np.zeros_like(pos)
    lib().orc_coordination(_p(pos), pos.shape[0], _p(a), a.size, _p(b), b.size, float(r0), int(n), int(m),
                           float(rcut), _p(L), int(bool(normalize)), _p(cn), _p(g))
    return float(cn[0]), g


def hillsum(xi, centers, heights, sigma, period):
    """O4: V(xi) and dV/dxi for Gaussian hills (centers K x D)."""
    xi = _f64(xi).reshape(-1)
    D = xi.size
    centers = _f64(centers).reshape(-1, D)
    heights = _f64(heights).reshape(-1)
    sigma = _f64(sigma).reshape(D)
    period = _f64(period).reshape(D)
    V = np.zeros(1)
    dV = np.zeros(D)
    lib().orc_hillsum(D, _p(xi), centers.shape[0], _p(centers), _p(heights), _p(sigma), _p(period), _p(V),
                      _p(dV))
    return float(V[0]), dV


def hillsum_batch(xi, hill_off, centers, heights, sigma, period, nthreads=1):
    """O4 over walkers: xi (W x D); hill_off (W+1) or None for shared hills."""
    xi = _f64(xi)
    W, D = xi.shape
    centers = _f64(centers).reshape(-1, D)
    heights = _f64(heights).reshape(-1)
    off = None if hill_off is None else np.ascontiguousarray(hill_off, dtype=np.int64)
    V = np.zeros(W)
    dV = np.zeros((W, D))
    lib().orc_hillsum_batch(W, D, _p(xi), _p(off), centers.shape[0], _p(centers), _p(heights),
                            _p(_f64(sigma)), _p(_f64(period)), _p(V), _p(dV), int(nthreads))
    return V, dV


def wt_height(w, V, kdT):
    """O5: well-tempered height w exp(-V/(k_B dT)); kdT <= 0 or inf: w."""
    return float(lib().orc_wt_height(float(w), float(V), float(kdT)))


def wt_sequence(centers, w, kdT, sigma, period, round_f32=True):
    """O5: heights of hills deposited one after another at the given centres."""
    centers = _f64(centers)
    K, D = centers.shape
    h = np.zeros(K)
    lib().orc_wt_sequence(D, K, _p(centers), float(w), float(kdT), _p(_f64(sigma)), _p(_f64(period)),
                          int(bool(round_f32)), _p(h))
    return h
