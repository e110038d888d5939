"""Python face of libsampx: a context object over the C ABI.

PyTorch supplies device memory and the stream; every step of the biasing
path runs in the library's HIP kernels.  Tensors passed to the hot-path
methods must already live on the context's device; nothing is copied.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import SX_AOS3, SX_AOS4, SX_F32, SX_F64, SX_SOA, SX_STEP_DEVICE, SxError  # noqa: F401

_LAYOUTS = {"aos3": SX_AOS3, "aos4": SX_AOS4, "soa": SX_SOA}


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _pos_dtype(t):
    if t.dtype == torch.float32:
        return SX_F32
    if t.dtype == torch.float64:
        return SX_F64
    raise TypeError("positions must be float32 or float64")


class Sampler:
    """One sampling context: CVs, walkers, a method, bound device state.

    Follows the initialize / update split of a PySAGES sampling method
    (Sec. 2.1): the definition calls and :meth:`bind` are the initialize
    step; :meth:`step` is the update that adds the biasing forces.
    """

    def __init__(self, device=0, stream=None):
        self.L = _lib.load()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        self._check(self.L.sx_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream)), None)
        self.h = h
        self.state = None
        self.ws = None
        self.n_walkers = 1
        self._per = []  # periodicity of each CV as added (dihedrals)
        self.n_atoms = None

    # ------------------------------------------------------------ plumbing
    def _check(self, st, h="self"):
        if st != 0:
            msg = ""
            if h == "self" and getattr(self, "h", None):
                msg = self.L.sx_last_error(self.h).decode()
            raise SxError(st, msg)

    def close(self):
        if getattr(self, "h", None):
            self.L.sx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self.stream = stream
        self._check(self.L.sx_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)))

    # --------------------------------------------------------------- CVs
    def add_dihedral(self, idx):
        a, p = _host(idx, np.int32)
        assert a.size == 4
        self._check(self.L.sx_add_cv_dihedral(self.h, p))
        self._per.append(True)

    def add_gyration(self, idx):
        a, p = _host(idx, np.int32)
        self._check(self.L.sx_add_cv_gyration(self.h, p, a.size))
        self._per.append(False)

    def add_coordination(self, a, b, r0, n=6, m=12, rcut=0.0, normalize=False):
        aa, pa = _host(a, np.int32)
        bb, pb = _host(b, np.int32)
        self._check(self.L.sx_add_cv_coordination(self.h, pa, aa.size, pb, bb.size, float(r0), int(n), int(m),
                                                  float(rcut), int(bool(normalize))))
        self._per.append(False)

    def _periodic(self):
        return list(self._per)

    def add_cvs(self, cvs):
        """Add CVs from the dict description used by the synthetic inputs."""
        for c in cvs:
            if c["kind"] == "dihedral":
                self.add_dihedral(c["idx"])
            elif c["kind"] == "gyration":
                self.add_gyration(c["idx"])
            elif c["kind"] == "coordination":
                self.add_coordination(c["a"], c["b"], c["r0"], c["n"], c["m"], c.get("rcut", 0.0),
                                      c.get("normalize", False))
            else:
                raise ValueError(c["kind"])

    def set_cell_lists(self, mode):
        """-1 never, 0 for large groups (default), 1 whenever the box allows."""
        self._check(self.L.sx_set_cell_lists(self.h, int(mode)))

    def cell_list_cvs(self):
        return int(self.L.sx_cell_list_cvs(self.h))

    def set_box(self, L):
        a, p = _host(L, np.float64)
        self._check(self.L.sx_set_box(self.h, p))

    @property
    def n_cvs(self):
        return int(self.L.sx_num_cvs(self.h))

    # ----------------------------------------------------------- walkers
    def set_walkers(self, atom_off, hill_capacity=None, shared=False):
        off, po = _host(atom_off, np.int64)
        cap = None
        pc = None
        if hill_capacity is not None:
            cap, pc = _host(hill_capacity, np.int64)
        self._check(self.L.sx_set_walkers(self.h, off.size - 1, po, pc, int(bool(shared))))
        self.n_walkers = off.size - 1
        self.n_atoms = int(off[-1])
        self._cap_keep = cap

    # ------------------------------------------------------------ methods
    def metad(self, sigma, height, temperature=300.0, bias_factor=None, stride=500, capacity=4096):
        s, p = _host(sigma, np.float64)
        bf = 0.0 if bias_factor is None else float(bias_factor)
        self._check(self.L.sx_metad_config(self.h, p, float(height), float(temperature), bf, int(stride),
                                           int(capacity)))

    def metad_dT(self, sigma, height, delta_T, stride=500, capacity=4096):
        s, p = _host(sigma, np.float64)
        self._check(self.L.sx_metad_config_dT(self.h, p, float(height), float(delta_T), int(stride), int(capacity)))

    def funn_fit(self, walker=0, batch=4096, steps=2000, lr=3e-3, lr_final=1e-5):
        """Fit the network to a walker's ABF mean forces (see sx_funn_fit);
        returns (visited bins used, final loss)."""
        n, loss = ctypes.c_int64(), ctypes.c_double()
        self._check(self.L.sx_funn_fit(self.h, int(walker), int(batch), int(steps), float(lr), float(lr_final),
                                       ctypes.byref(n), ctypes.byref(loss)))
        return n.value, loss.value

    def funn_enable(self, on=True):
        self._check(self.L.sx_funn_enable(self.h, int(bool(on))))

    def abf_momentum(self, dt, masses):
        """Use the momentum-derivative ABF estimator (see sx_abf_momentum);
        step() then takes the momenta as sys_forces."""
        m, pm = _host(masses, np.float64)
        self._check(self.L.sx_abf_momentum(self.h, float(dt), pm, m.size))

    def metad_fes(self, lo, hi, nbins, temperature=300.0, walker=0):
        """Free energy of the metadynamics bias at the nodes of an analysis
        grid (per CV nbins nodes over a periodic range, nbins + 1 up to hi
        otherwise; row-major), shifted to min 0; host array of the grid's
        shape.  See sx_fes_metad_grid."""
        D = self.D
        l, pl = _host(lo, np.float64)
        h, ph = _host(hi, np.float64)
        nb, pn = _host(nbins, np.int32)
        nodes = np.zeros(D, dtype=np.int32)
        pnodes = nodes.ctypes.data_as(ctypes.c_void_p)
        self._check(self.L.sx_fes_metad_grid(self.h, int(walker), pl, ph, pn, float(temperature), pnodes, None, 0))
        F = np.empty(int(np.prod(nodes)), dtype=np.float64)
        self._check(self.L.sx_fes_metad_grid(self.h, int(walker), pl, ph, pn, float(temperature), pnodes,
                                             F.ctypes.data_as(ctypes.c_void_p), F.size))
        return F.reshape([int(k) for k in nodes])

    def abf_fes(self, walker=0):
        """Free energy at the ABF bin centres (see sx_abf_fes): host array of
        the grid's shape, NaN at unvisited bins."""
        A = np.empty(int(np.prod(self.nbins)))
        self._check(self.L.sx_abf_fes(self.h, int(walker), A.ctypes.data_as(ctypes.c_void_p)))
        return A.reshape(self.nbins)

    def harmonic(self, k, centers):
        """Harmonic bias with one window centre per walker (centers: W x D)."""
        k_, pk = _host(k, np.float64)
        c, pc = _host(centers, np.float64)
        self._check(self.L.sx_harmonic_config(self.h, pk, pc, int(c.reshape(-1, k_.size).shape[0])))

    def umbrella_reset(self):
        self._check(self.L.sx_umbrella_reset(self.h))

    def umbrella_stats(self):
        """(samples (W,), means (W, D), covariances (W, D, D)), host."""
        W, D = self.n_walkers, self.D
        n = np.zeros(W, dtype=np.int64)
        m = np.zeros((W, D))
        c = np.zeros((W, D, D))
        self._check(self.L.sx_umbrella_stats(self.h, n.ctypes.data_as(ctypes.c_void_p),
                                             m.ctypes.data_as(ctypes.c_void_p), c.ctypes.data_as(ctypes.c_void_p)))
        return n, m, c

    def umbrella_integrate(self):
        """(mean forces (W, D), A (W,)) by umbrella integration along the
        windows in walker order."""
        W, D = self.n_walkers, self.D
        g = np.zeros((W, D))
        A = np.zeros(W)
        self._check(self.L.sx_umbrella_integrate(self.h, g.ctypes.data_as(ctypes.c_void_p),
                                                 A.ctypes.data_as(ctypes.c_void_p)))
        return g, A

    def metad_grid(self, lo, hi, nbins):
        """Keep the metadynamics bias on a grid (see sx_metad_grid); pass
        None for all three to switch it off."""
        if lo is None and hi is None and nbins is None:
            self._check(self.L.sx_metad_grid(self.h, None, None, None))
            return
        lo_, plo = _host(lo, np.float64)
        hi_, phi = _host(hi, np.float64)
        nb, pn = _host(nbins, np.int32)
        self._check(self.L.sx_metad_grid(self.h, plo, phi, pn))

    def abf(self, lo, hi, nbins, n_threshold=500):
        lo_, plo = _host(lo, np.float64)
        hi_, phi = _host(hi, np.float64)
        nb, pn = _host(nbins, np.int32)
        self._check(self.L.sx_abf_config(self.h, plo, phi, pn, int(n_threshold)))
        self.nbins = [int(x) for x in nb]

    # ------------------------------------------------------------ binding
    def bind(self):
        sb = int(self.L.sx_state_bytes(self.h))
        wb = int(self.L.sx_workspace_bytes(self.h))
        if sb == 0 or wb == 0:  # the plan failed: sx_bind reports why
            self._check(self.L.sx_bind(self.h, None, 0, None, 0))
            self._check(_lib.SX_ESTATE)
        # torch's caching allocator returns 512-byte aligned blocks
        self.state = torch.empty(sb, dtype=torch.uint8, device=self.device)
        self.ws = torch.empty(wb, dtype=torch.uint8, device=self.device)
        self._check(self.L.sx_bind(self.h, _ptr(self.state), sb, _ptr(self.ws), wb))
        self.D = self.n_cvs
        self.n_slots = int(self.L.sx_jac_slots(self.h))
        return sb, wb

    # ----------------------------------------------------------- hot path
    def step(self, pos, forces=None, step=None, xi_out=None, V_out=None, dV_out=None, sys_forces=None,
             layout="aos3"):
        st = SX_STEP_DEVICE if step is None else int(step)
        self._check(self.L.sx_step(self.h, _ptr(pos), _pos_dtype(pos), _LAYOUTS[layout], st, _ptr(xi_out),
                                   _ptr(V_out), _ptr(dV_out), _ptr(forces), _ptr(sys_forces)))

    def check(self):
        self._check(self.L.sx_check(self.h))

    def eval_cv(self, pos, jac=True, layout="aos3"):
        W = self.n_walkers
        xi = torch.empty((W, self.D), dtype=torch.float64, device=self.device)
        J = torch.empty((W, self.n_slots, 3), dtype=torch.float32, device=self.device) if jac else None
        self._check(self.L.sx_eval_cv(self.h, _ptr(pos), _pos_dtype(pos), _LAYOUTS[layout], _ptr(xi), _ptr(J)))
        return xi, J

    def jac_layout(self):
        n = self.n_slots
        atom = np.zeros(n, dtype=np.int32)
        cv = np.zeros(n, dtype=np.int32)
        self._check(self.L.sx_jac_layout(self.h, atom.ctypes.data_as(ctypes.c_void_p),
                                         cv.ctypes.data_as(ctypes.c_void_p)))
        return atom, cv

    def cv_vjp(self, pos, xi_bar, pos_bar, layout="aos3"):
        self._check(self.L.sx_cv_vjp(self.h, _ptr(pos), _pos_dtype(pos), _LAYOUTS[layout], _ptr(xi_bar),
                                     _ptr(pos_bar)))

    def hillsum(self, xi):
        W = self.n_walkers
        V = torch.empty(W, dtype=torch.float64, device=self.device)
        dV = torch.empty((W, self.D), dtype=torch.float64, device=self.device)
        self._check(self.L.sx_hillsum(self.h, _ptr(xi), _ptr(V), _ptr(dV)))
        return V, dV

    def bias_eval(self, xi, walker=0, grad=True):
        """Bias V and dV/dxi of a hill list at query points xi (n x D, device
        float64): the step's arithmetic at arbitrary points."""
        n = xi.shape[0]
        V = torch.empty(n, dtype=torch.float64, device=self.device)
        dV = torch.empty((n, self.D), dtype=torch.float64, device=self.device) if grad else None
        self._check(self.L.sx_bias_eval(self.h, int(walker), _ptr(xi.contiguous()), n, _ptr(V), _ptr(dV)))
        return V, dV

    def bias_eval_noalloc(self, xi, V, dV=None, walker=0):
        """bias_eval into caller-given outputs V (n) and dV (n x D, or None),
        through the entry point that allocates nothing (its partial sums in
        the library's fixed scratch)."""
        self._check(self.L.sx_bias_eval_noalloc(self.h, int(walker), _ptr(xi), xi.shape[0], _ptr(V), _ptr(dV)))

    def grid_eval(self, xi, walker=0, grad=True):
        """The bias grid's read-back (multilinear interpolation) at points xi
        (n x D, device float64)."""
        n = xi.shape[0]
        V = torch.empty(n, dtype=torch.float64, device=self.device)
        dV = torch.empty((n, self.D), dtype=torch.float64, device=self.device) if grad else None
        self._check(self.L.sx_grid_eval(self.h, int(walker), _ptr(xi.contiguous()), n, _ptr(V), _ptr(dV)))
        return V, dV

    def grid_get(self, walker=0):
        """Node values of a bias grid: V (nodes,) and dV/dxi (D, nodes), host
        float64, nodes row-major (first CV slowest)."""
        n = int(self.L.sx_grid_nodes(self.h))
        V = np.empty(n)
        G = np.empty((self.D, n))
        self._check(self.L.sx_grid_get(self.h, int(walker), V.ctypes.data_as(ctypes.c_void_p),
                                       G.ctypes.data_as(ctypes.c_void_p), n))
        return V, G

    def deposit(self, xi):
        self._check(self.L.sx_deposit(self.h, _ptr(xi)))

    # ------------------------------------------------------------ state I/O
    def hills_set(self, walker, centers, heights):
        c, pc = _host(centers, np.float32)
        h, ph = _host(heights, np.float32)
        self._check(self.L.sx_hills_set(self.h, int(walker), pc, ph, h.size))

    def hills_get(self, walker, max_k=None):
        K = ctypes.c_int64()
        self._check(self.L.sx_hills_get(self.h, int(walker), None, None, 0, ctypes.byref(K)))
        n = K.value if max_k is None else min(K.value, max_k)
        c = np.zeros((n, self.D), dtype=np.float32)
        h = np.zeros(n, dtype=np.float32)
        self._check(self.L.sx_hills_get(self.h, int(walker), c.ctypes.data_as(ctypes.c_void_p),
                                        h.ctypes.data_as(ctypes.c_void_p), n, ctypes.byref(K)))
        return c, h

    def hill_counts(self):
        """Number of hills in each walker's list (host copy, synchronous)."""
        out = np.zeros(self.n_walkers, dtype=np.int64)
        K = ctypes.c_int64()
        for w in range(self.n_walkers):
            self._check(self.L.sx_hills_get(self.h, w, None, None, 0, ctypes.byref(K)))
            out[w] = K.value
        return out

    def abf_grid(self, walker=0):
        nb = int(np.prod(self.nbins))
        N = np.zeros(nb, dtype=np.uint32)
        F = np.zeros((nb, self.D), dtype=np.float64)
        self._check(self.L.sx_abf_grid_get(self.h, int(walker), N.ctypes.data_as(ctypes.c_void_p),
                                           F.ctypes.data_as(ctypes.c_void_p)))
        return N, F

    def get_step(self):
        s = ctypes.c_int64()
        self._check(self.L.sx_get_step(self.h, ctypes.byref(s)))
        return s.value

    def export_state(self):
        n = int(self.L.sx_checkpoint_bytes(self.h))
        buf = np.zeros(n, dtype=np.uint8)
        self._check(self.L.sx_state_export(self.h, buf.ctypes.data_as(ctypes.c_void_p), n))
        return buf

    def import_state(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self.L.sx_state_import(self.h, buf.ctypes.data_as(ctypes.c_void_p), buf.size))

    # ------------------------------------------------------------ surrogate
    def surrogate(self, hidden=64, max_samples=1 << 17, max_batch=4096, cert_n=512, tol_force=0.1):
        """Declare the bias surrogate network (before bind)."""
        self._check(self.L.sx_surrogate_config(self.h, int(hidden), int(max_samples), int(max_batch), int(cert_n),
                                               float(tol_force)))

    def surrogate_norm(self, mu, s):
        m, pm = _host(mu, np.float64)
        s_, ps = _host(s, np.float64)
        self._check(self.L.sx_surrogate_norm(self.h, pm, ps))

    def surrogate_param_count(self):
        return int(self.L.sx_surrogate_param_count(self.h))

    def surrogate_params(self, params=None):
        """Set (params given, host float32 vector of length P) or get them."""
        n = self.surrogate_param_count()
        if params is not None:
            a, pa = _host(params, np.float32)
            self._check(self.L.sx_surrogate_params_set(self.h, pa, a.size))
            return None
        out = np.zeros(n, dtype=np.float32)
        self._check(self.L.sx_surrogate_params_get(self.h, out.ctypes.data_as(ctypes.c_void_p), n))
        return out

    def surrogate_output(self, scale=None, shift=None):
        if scale is not None:
            self._check(self.L.sx_surrogate_output(self.h, float(scale), float(shift)))
            return None
        a, b = ctypes.c_double(), ctypes.c_double()
        self._check(self.L.sx_surrogate_output_get(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def surrogate_eval(self, xi, fallback=False):
        n = xi.shape[0]
        V = torch.empty(n, dtype=torch.float64, device=self.device)
        dV = torch.empty((n, self.D), dtype=torch.float64, device=self.device)
        fb = torch.empty(n, dtype=torch.uint8, device=self.device) if fallback else None
        self._check(self.L.sx_surrogate_eval(self.h, _ptr(xi.contiguous()), n, _ptr(V), _ptr(dV), _ptr(fb)))
        return (V, dV, fb) if fallback else (V, dV)

    def surrogate_loss_grad(self, xi, V, G, alpha, beta):
        n = xi.shape[0]
        g = np.zeros(self.surrogate_param_count(), dtype=np.float64)
        loss = ctypes.c_double()
        self._check(self.L.sx_surrogate_loss_grad(self.h, _ptr(xi.contiguous()), _ptr(V.contiguous()),
                                                  _ptr(G.contiguous()), n, float(alpha), float(beta),
                                                  g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss)))
        return loss.value, g

    def surrogate_fit(self, xi, V, G, batch, steps, lr, lr_final=0.0, alpha=1.0, beta=1.0):
        loss = ctypes.c_double()
        self._check(self.L.sx_surrogate_fit(self.h, _ptr(xi.contiguous()), _ptr(V.contiguous()), _ptr(G.contiguous()),
                                            xi.shape[0], int(batch), int(steps), float(lr), float(lr_final),
                                            float(alpha), float(beta), ctypes.byref(loss)))
        return loss.value

    def surrogate_train(self, xi, batch=4096, steps=20000, lr=3e-3, lr_final=1e-5):
        loss = ctypes.c_double()
        self._check(self.L.sx_surrogate_train(self.h, _ptr(xi.contiguous()), xi.shape[0], int(batch), int(steps),
                                              float(lr), float(lr_final), ctypes.byref(loss)))
        return loss.value

    def surrogate_certify(self, lo=None, hi=None):
        frac = ctypes.c_double()
        plo = _host(lo, np.float64) if lo is not None else (None, None)
        phi = _host(hi, np.float64) if hi is not None else (None, None)
        self._check(self.L.sx_surrogate_certify(self.h, plo[1], phi[1], ctypes.byref(frac)))
        return frac.value

    def surrogate_tolerance(self, tol_force):
        self._check(self.L.sx_surrogate_tolerance(self.h, float(tol_force)))

    def surrogate_enable(self, on=True):
        self._check(self.L.sx_surrogate_enable(self.h, 1 if on else 0))

    def surrogate_fallback_count(self):
        c = ctypes.c_int32()
        self._check(self.L.sx_surrogate_fallback_count(self.h, ctypes.byref(c)))
        return c.value

    # ----------------------------------------------------- graphs / tuning
    def graph_capture(self, n_steps, pos, forces=None, xi_out=None, V_out=None, dV_out=None, sys_forces=None,
                      layout="aos3"):
        self._check(self.L.sx_graph_capture(self.h, int(n_steps), _ptr(pos), _pos_dtype(pos), _LAYOUTS[layout],
                                            _ptr(xi_out), _ptr(V_out), _ptr(dV_out), _ptr(forces),
                                            _ptr(sys_forces)))

    def graph_launch(self):
        self._check(self.L.sx_graph_launch(self.h))

    def set_tuning(self, tile_hills, grid=0):
        self._check(self.L.sx_set_tuning(self.h, int(tile_hills), int(grid)))

    def get_tuning(self):
        t = ctypes.c_int32()
        g = ctypes.c_int32()
        self._check(self.L.sx_get_tuning(self.h, ctypes.byref(t), ctypes.byref(g)))
        return t.value, g.value

    def time_cell(self, pos, forces=None, reps=20, layout="aos3"):
        """ms per launch of the cell sort, the pair pass and the VJP gather
        (graph-replayed launches; the measurement library's sx_time_cell)."""
        a, b, c = ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
        M = _lib.load_measure()
        self._check(M.sx_time_cell(self.h, _ptr(pos), _pos_dtype(pos), _LAYOUTS[layout], _ptr(forces), int(reps),
                                   ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def time_hill(self, pos, forces=None, reps=100, layout="aos3"):
        """(ms per tile-kernel launch, ms per finalize-kernel launch): `reps`
        launches of each captured in a graph and replayed between hipEvents
        on the context's stream (the measurement library's sx_time_hill)."""
        m1, m2 = ctypes.c_float(), ctypes.c_float()
        M = _lib.load_measure()
        self._check(M.sx_time_hill(self.h, _ptr(pos), _pos_dtype(pos), _LAYOUTS[layout], _ptr(forces), int(reps),
                                   ctypes.byref(m1), ctypes.byref(m2)))
        return m1.value, m2.value

    def time_hill_step(self, pos, forces=None, reps=100, layout="aos3"):
        """(ms per (tile kernel, finalize kernel) pair in a graph, ms per
        launch of a graph of empty one-workgroup kernels): see
        sx_time_hill_step."""
        m1, m2 = ctypes.c_float(), ctypes.c_float()
        M = _lib.load_measure()
        self._check(M.sx_time_hill_step(self.h, _ptr(pos), _pos_dtype(pos), _LAYOUTS[layout], _ptr(forces), int(reps),
                                        ctypes.byref(m1), ctypes.byref(m2)))
        return m1.value, m2.value

    def autotune(self, pos=None, cache_path=None, layout="aos3"):
        """Pick the hill-sum tiling by timing the step's kernels (see sx_autotune)."""
        dt = 0 if pos is None else _pos_dtype(pos)
        self._check(self.L.sx_autotune(self.h, _ptr(pos), dt, _LAYOUTS[layout],
                                       None if cache_path is None else cache_path.encode()))
