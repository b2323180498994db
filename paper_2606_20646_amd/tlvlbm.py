"""Python binding of the tlvlbm C ABI (``include/tlvlbm.h``).

Argument marshalling only: every step of the method runs in the HIP kernels of
``libtlvlbm.so``.  Arrays may be numpy (host) or torch tensors (host or
device); device tensors are passed by pointer.  The library must have been
built (``paper_2606_20646_amd.build``); importing this module without it
raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TLVLBM_LIBRARY") or os.path.join(HERE, "libtlvlbm.so")

OK, ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_NONPOSITIVE_J, ERR_NEWTON, ERR_NONFINITE, \
    ERR_CALL_ORDER = range(8)
FP32, FP64 = 0, 1
DIRICHLET, NEUMANN = 1, 2
RAMPS = {"const": 0, "sin2": 1, "halfcos": 2, "linear": 3}


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("dx", C.c_double), ("origin", C.c_double * 3),
                ("periodic_mask", C.c_uint32)]


class Material(C.Structure):
    _fields_ = [("law", C.c_int32), ("mu", C.c_double), ("lam", C.c_double), ("k1", C.c_double),
                ("a0", C.c_double * 3), ("beta", C.c_double), ("tau", C.c_double)]


def _material(mu, lam, fibre, viscous=None):
    """law 0 (neo-Hookean); with fibre = (k1, a0), law 1; with viscous =
    (beta, tau), law 2 (a Maxwell branch, on top of the fibres if given)."""
    m = Material(0, mu, lam, 0.0)
    if fibre is not None:
        k1, a0 = fibre
        m.law, m.k1 = 1, float(k1)
        for k, v in enumerate(a0):
            m.a0[k] = v
    if viscous is not None:
        m.law = 2
        m.beta, m.tau = float(viscous[0]), float(viscous[1])
    return m


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Options(C.Structure):
    _fields_ = [("omega", C.c_double), ("gamma", C.c_double), ("theta_F", C.c_double), ("cg_rtol", C.c_double),
                ("proj_every", C.c_int32), ("cg_maxit", C.c_int32), ("precision", C.c_int32),
                ("track_u", C.c_int32), ("stream", C.c_void_p), ("cg_multigrid", C.c_int32),
                ("proj_sweeps", C.c_int32), ("proj_weight", C.c_double), ("dev_alloc", ALLOC_FN),
                ("dev_free", FREE_FN), ("alloc_user", C.c_void_p)]


def torch_allocator(stream=None):
    """(dev_alloc, dev_free) callbacks that hand the library's device memory
    to torch's caching allocator (torch.cuda.caching_allocator_alloc /
    _delete) on the current device, associated with `stream` (a
    torch.cuda.Stream; None: the current stream)."""
    import torch
    dev = torch.cuda.current_device()

    def alloc(nbytes, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
        except Exception:  # out of memory: the library reports TLVLBM_ERR_OUT_OF_MEMORY
            return None

    def free(ptr, user):
        torch.cuda.caching_allocator_delete(ptr)

    return ALLOC_FN(alloc), FREE_FN(free)


class BC(C.Structure):
    _fields_ = [("type", C.c_int32), ("ramp", C.c_int32), ("T_r", C.c_double),
                ("given_as_displacement", C.c_int32), ("a", C.c_double * 3), ("G", C.c_double * 9),
                ("p_radial", C.c_double), ("p_normal", C.c_double), ("X0", C.c_double * 3),
                ("twist", C.c_double)]


class Stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("active_nodes", "cut_links", "dirichlet_links", "neumann_links",
                                         "cg_iterations", "newton_failures", "projections", "step",
                                         "lsq_linear_fallbacks")]


class TlvlbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tlvlbm error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_20646_amd.build`")
    # One HIP runtime per process: when PyTorch is installed it must be loaded
    # first, so that the library binds to the runtime PyTorch ships (whose
    # streams and device pointers callers pass in).  Loading the system
    # runtime first leaves PyTorch without devices.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, dp = C.c_void_p, C.c_void_p
    L.tlvlbm_default_options.argtypes = [C.POINTER(Options)]
    L.tlvlbm_create.argtypes = [C.POINTER(Grid), C.c_int, C.POINTER(Material), C.c_double, C.c_double,
                                C.POINTER(Options), C.POINTER(vp)]
    L.tlvlbm_destroy.argtypes = [vp]
    L.tlvlbm_set_levelset.argtypes = [vp, dp, dp]
    L.tlvlbm_set_boundary.argtypes = [vp, C.c_uint8, C.POINTER(BC)]
    L.tlvlbm_set_material.argtypes = [vp, C.POINTER(Material)]
    L.tlvlbm_set_body_force.argtypes = [vp, C.c_void_p, C.c_int32, C.c_double]
    L.tlvlbm_set_thermal_stretch.argtypes = [vp, C.c_void_p]
    L.tlvlbm_set_state.argtypes = [vp, dp, dp, dp]
    L.tlvlbm_step.argtypes = [vp, C.c_int64]
    L.tlvlbm_moments.argtypes = [vp, dp, dp, dp]
    L.tlvlbm_stress.argtypes = [vp, dp, dp]
    L.tlvlbm_moments_native.argtypes = [vp, dp, dp, dp]
    L.tlvlbm_get_history.argtypes = [vp, dp]
    L.tlvlbm_put_history.argtypes = [vp, dp]
    L.tlvlbm_get_state.argtypes = [vp, dp, dp, C.POINTER(C.c_int64)]
    L.tlvlbm_put_state.argtypes = [vp, dp, dp, C.c_int64]
    L.tlvlbm_get_links.argtypes = [vp, dp, dp, dp, dp, dp]
    L.tlvlbm_stats.argtypes = [vp, C.POINTER(Stats)]
    L.tlvlbm_synchronize.argtypes = [vp]
    L.tlvlbm_last_error.argtypes = [vp]
    L.tlvlbm_last_error.restype = C.c_char_p
    L.tlvlbm_population_bytes.argtypes = [vp]
    L.tlvlbm_population_bytes.restype = C.c_size_t
    L.tlvlbm_step_each.argtypes = [C.POINTER(vp), C.c_int32, C.c_int64]
    L.tlvlbm_adjoint_step.argtypes = [vp, C.c_int64, dp, dp, dp, dp, C.POINTER(C.c_double), dp, dp, C.c_int64]
    L.tlvlbm_adjoint_record.argtypes = [vp, C.c_int64, dp, dp, C.c_int64]
    L.tlvlbm_adjoint_backward.argtypes = [vp, dp, dp, C.POINTER(C.c_double), dp, dp, dp]
    L.tlvlbm_cut_links_noalloc.argtypes = [C.POINTER(Grid), C.c_int, dp, dp, C.c_int64, dp, dp, dp, dp, dp,
                                           C.POINTER(C.c_int64), vp]
    L.tlvlbm_cut_links_noalloc.restype = C.c_int
    L.tlvlbm_batch_create.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(vp)]
    L.tlvlbm_batch_step.argtypes = [vp, C.c_int64]
    L.tlvlbm_batch_set_graph.argtypes = [vp, C.c_int32]
    L.tlvlbm_batch_autotune.argtypes = [vp, C.c_int32]
    L.tlvlbm_batch_set_tiles.argtypes = [vp, C.c_int32, C.c_int32]
    L.tlvlbm_batch_get_tiles.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    L.tlvlbm_batch_destroy.argtypes = [vp]
    L.tlvlbm_batch_last_error.argtypes = [vp]
    L.tlvlbm_batch_last_error.restype = C.c_char_p
    for name in ("create", "destroy", "set_levelset", "set_boundary", "set_material", "set_state", "step",
                 "moments", "get_state", "put_state", "get_links", "stats", "synchronize", "step_each",
                 "batch_create", "batch_step", "batch_set_graph", "batch_destroy", "adjoint_step",
                 "adjoint_record", "adjoint_backward",
                 "batch_autotune", "batch_set_tiles", "batch_get_tiles"):
        getattr(L, "tlvlbm_" + name).restype = C.c_int
    return L


lib = _load()


def _ptr(a):
    """(pointer, keepalive) for numpy arrays and torch tensors (contiguous)."""
    if a is None:
        return None, None
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            a = np.ascontiguousarray(a)
        return a.ctypes.data, a
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor arguments must be contiguous")
        return a.data_ptr(), a
    raise TypeError(f"unsupported array type {type(a)}")


class Solver:
    """One TL-VLBM lattice on the GPU (see include/tlvlbm.h for semantics)."""

    def __init__(self, D, n, dx, dt, mu, lam, rho0=1.0, origin=None, periodic_mask=None, omega=1.8, gamma=0.0,
                 theta_F=1.0, proj_every=20, precision="fp32", track_u=-1, cg_rtol=0.0, cg_maxit=0,
                 stream=None, cg_multigrid=True, proj_sweeps=20, proj_weight=2.0 / 3.0, fibre=None,
                 allocator=None, viscous=None):
        """allocator: None (the library's hipMalloc), "torch" (torch's caching
        allocator, on the stream given as a torch.cuda.Stream or the current
        one), or a (dev_alloc, dev_free) pair of ALLOC_FN / FREE_FN.
        fibre = (k1, a0): fibre-reinforced law; viscous = (beta, tau): one
        Maxwell branch (tau = inf: glassy limit)."""
        self.D, self.M, self.Q = D, D + D * D, 2 * D
        self.n = tuple(int(v) for v in n)
        self.N = int(np.prod(self.n))
        self.dx, self.dt = float(dx), float(dt)
        g = Grid()
        for a in range(3):
            g.n[a] = self.n[a] if a < D else 1
            g.origin[a] = (origin[a] if origin is not None and a < len(origin) else 0.0)
        g.dx = dx
        g.periodic_mask = ((1 << D) - 1) if periodic_mask is None else periodic_mask
        m = _material(mu, lam, fibre, viscous)
        o = Options()
        lib.tlvlbm_default_options(C.byref(o))
        o.omega, o.gamma, o.theta_F, o.cg_rtol = omega, gamma, theta_F, cg_rtol
        o.proj_every, o.cg_maxit, o.track_u = proj_every, cg_maxit, track_u
        o.precision = FP64 if precision in ("fp64", FP64) else FP32
        self.precision = o.precision
        tstream = None
        if stream is not None and hasattr(stream, "cuda_stream"):  # a torch.cuda.Stream
            tstream, stream = stream, stream.cuda_stream
        o.stream = stream
        self._alloc = None
        if allocator == "torch":
            self._alloc = torch_allocator(tstream)
        elif allocator is not None:
            self._alloc = tuple(allocator)
        if self._alloc is not None:
            o.dev_alloc, o.dev_free = self._alloc
        o.cg_multigrid = int(bool(cg_multigrid))
        o.proj_sweeps, o.proj_weight = int(proj_sweeps), float(proj_weight)
        h = C.c_void_p()
        st = lib.tlvlbm_create(C.byref(g), D, C.byref(m), rho0, dt, C.byref(o), C.byref(h))
        if st:
            raise TlvlbmError(st, "create failed")
        self.h = h

    def close(self):
        # at interpreter exit the module globals may already be gone
        if getattr(self, "h", None) and lib is not None:
            lib.tlvlbm_destroy(self.h)
            self.h = None

    __del__ = close

    def _chk(self, st, what):
        if st:
            raise TlvlbmError(st, f"{what}: {lib.tlvlbm_last_error(self.h).decode()}")

    def set_levelset(self, phi, bid=None):
        phi = phi if not isinstance(phi, np.ndarray) else np.ascontiguousarray(phi, np.float64).reshape(-1)
        bid = bid if (bid is None or not isinstance(bid, np.ndarray)) else np.ascontiguousarray(bid, np.uint8)
        p1, k1 = _ptr(phi)
        p2, k2 = _ptr(bid)
        self._chk(lib.tlvlbm_set_levelset(self.h, p1, p2), "set_levelset")

    def set_boundary(self, bid, type, ramp="const", T_r=1.0, given_as_displacement=False, a=None, G=None,
                     p_radial=0.0, p_normal=0.0, X0=None, twist=0.0):
        b = BC()
        b.type = {"dirichlet": DIRICHLET, "neumann": NEUMANN}.get(type, type)
        b.ramp = RAMPS.get(ramp, ramp)
        b.T_r = T_r
        b.given_as_displacement = int(bool(given_as_displacement))
        for k, v in enumerate(a if a is not None else []):
            b.a[k] = v
        if G is not None:
            G = np.asarray(G, float)
            for i in range(G.shape[0]):
                for j in range(G.shape[1]):
                    b.G[i * 3 + j] = G[i, j]
        b.p_radial, b.p_normal = p_radial, p_normal
        for k, v in enumerate(X0 if X0 is not None else []):
            b.X0[k] = v
        b.twist = float(twist)
        self._chk(lib.tlvlbm_set_boundary(self.h, int(bid), C.byref(b)), "set_boundary")

    def set_thermal_stretch(self, th):
        """Thermal stretch th [N] per node (> 0; numpy or device tensor; None
        removes it): P(F) = th^(D-1) P_W(F / th)."""
        arr = th if (th is None or not isinstance(th, np.ndarray)) else np.ascontiguousarray(th, np.float64)
        p, keep = _ptr(arr)
        self._chk(lib.tlvlbm_set_thermal_stretch(self.h, p), "set_thermal_stretch")

    def set_body_force(self, g, ramp="const", T_r=1.0):
        """Body acceleration b(X, t) = s(t) g(X); g [D][N] numpy or device
        tensor (None removes it)."""
        arr = g if (g is None or not isinstance(g, np.ndarray)) else np.ascontiguousarray(g, np.float64)
        p, keep = _ptr(arr)
        self._chk(lib.tlvlbm_set_body_force(self.h, p, RAMPS.get(ramp, ramp), float(T_r)), "set_body_force")

    def set_material(self, mu, lam, fibre=None, viscous=None):
        self._chk(lib.tlvlbm_set_material(self.h, C.byref(_material(mu, lam, fibre, viscous))), "set_material")

    def set_state(self, U0, u0=None, dU0=None):
        arrs = [a if (a is None or not isinstance(a, np.ndarray)) else np.ascontiguousarray(a, np.float64)
                for a in (U0, u0, dU0)]
        ptrs = [_ptr(a) for a in arrs]
        self._chk(lib.tlvlbm_set_state(self.h, ptrs[0][0], ptrs[1][0], ptrs[2][0]), "set_state")
        self._init = (arrs[0], arrs[2])  # the reverse mode transposes the initialisation

    def adjoint(self, n, dLdU=None, dLdu=None, segment=0, grad_v0=True, grad_u0=True):
        """Advance n steps from the state of set_state and return
        (dL/d(mu, lambda), dL/dv0 [D][N], dL/du0 [D][N]) for
        L = sum dLdU . U + dLdu . u over the moments after the last step.
        dLdU, dLdu: numpy arrays or contiguous float64 torch tensors (host or
        device).  grad_v0 / grad_u0: True (new numpy arrays), False (not
        computed) or a contiguous float64 tensor [D][N] to write into."""
        U0, dU0 = self._init
        gm = (C.c_double * 2)()

        def out(spec):
            if spec is True:
                return np.zeros((self.D, self.N))
            return spec if spec is not False and spec is not None else None

        gv, g0 = out(grad_v0), out(grad_u0)
        args = [a if (a is None or not isinstance(a, np.ndarray)) else np.ascontiguousarray(a, np.float64)
                for a in (dLdU, dLdu)]
        self._chk(lib.tlvlbm_adjoint_step(self.h, int(n), _ptr(U0)[0], _ptr(dU0)[0], _ptr(args[0])[0],
                                          _ptr(args[1])[0], gm, _ptr(gv)[0], _ptr(g0)[0], int(segment)), "adjoint")
        return np.array([gm[0], gm[1]]), gv, g0

    def adjoint_record(self, n, segment=0):
        """First pass of the reverse mode: n steps from the state of
        set_state with checkpoints and tape (tlvlbm_adjoint_record)."""
        U0, dU0 = self._init
        self._chk(lib.tlvlbm_adjoint_record(self.h, int(n), _ptr(U0)[0], _ptr(dU0)[0], int(segment)),
                  "adjoint_record")

    def adjoint_backward(self, dLdU=None, dLdu=None, grad_v0=True, grad_u0=True, grad_dU0=False):
        """Reverse pass of the recorded run (tlvlbm_adjoint_backward): returns
        (dL/d(mu, lambda), dL/dv0, dL/du0, dL/d dU0).  Output specs as in
        adjoint(); grad_dU0 True gives a new [D][M][N] numpy array."""
        gm = (C.c_double * 2)()

        def out(spec, shape):
            if spec is True:
                return np.zeros(shape)
            return spec if spec is not False and spec is not None else None

        gv, g0 = out(grad_v0, (self.D, self.N)), out(grad_u0, (self.D, self.N))
        gd = out(grad_dU0, (self.D, self.M, self.N))
        args = [a if (a is None or not isinstance(a, np.ndarray)) else np.ascontiguousarray(a, np.float64)
                for a in (dLdU, dLdu)]
        self._chk(lib.tlvlbm_adjoint_backward(self.h, _ptr(args[0])[0], _ptr(args[1])[0], gm, _ptr(gv)[0],
                                              _ptr(g0)[0], _ptr(gd)[0]), "adjoint_backward")
        return np.array([gm[0], gm[1]]), gv, g0, gd

    def step(self, n=1):
        self._chk(lib.tlvlbm_step(self.h, int(n)), "step")

    def moments(self, U=True, u=True, J=True):
        Uo = np.zeros((self.M, self.N)) if U else None
        uo = np.zeros((self.D, self.N)) if u else None
        Jo = np.zeros(self.N) if J else None
        self._chk(lib.tlvlbm_moments(self.h, _ptr(Uo)[0], _ptr(uo)[0], _ptr(Jo)[0]), "moments")
        return Uo, uo, Jo

    def moments_native(self):
        """(U [M][N], u [D][N], J [N]): U and J in the context's precision
        (float32 for FP32 contexts), u in float64"""
        dt = np.float64 if self.precision == FP64 else np.float32
        Uo = np.zeros((self.M, self.N), dt)
        uo = np.zeros((self.D, self.N))
        Jo = np.zeros(self.N, dt)
        self._chk(lib.tlvlbm_moments_native(self.h, _ptr(Uo)[0], _ptr(uo)[0], _ptr(Jo)[0]), "moments_native")
        return Uo, uo, Jo

    def stress(self, P=True, sigma=True):
        """(P, sigma) of the current time level, [D*D][N] each (Eq. 35)"""
        Po = np.zeros((self.D * self.D, self.N)) if P else None
        So = np.zeros((self.D * self.D, self.N)) if sigma else None
        self._chk(lib.tlvlbm_stress(self.h, _ptr(Po)[0], _ptr(So)[0]), "stress")
        return Po, So

    def moments_into(self, U=None, u=None, J=None):
        """Write moments into caller buffers (numpy or torch, host or device)."""
        self._chk(lib.tlvlbm_moments(self.h, _ptr(U)[0], _ptr(u)[0], _ptr(J)[0]), "moments")

    def get_state(self):
        f = np.zeros((self.Q, self.M, self.N))
        us = np.zeros((self.D, self.N))
        st = C.c_int64(0)
        self._chk(lib.tlvlbm_get_state(self.h, _ptr(f)[0], _ptr(us)[0], C.byref(st)), "get_state")
        return f, us, st.value

    def get_history(self):
        """the Maxwell branch's history R [D(D+1)/2][N] (law 2)"""
        R = np.zeros((self.D * (self.D + 1) // 2, self.N))
        self._chk(lib.tlvlbm_get_history(self.h, _ptr(R)[0]), "get_history")
        return R

    def put_history(self, R):
        R = np.ascontiguousarray(R, np.float64)
        self._chk(lib.tlvlbm_put_history(self.h, _ptr(R)[0]), "put_history")

    def put_state(self, f, ustar=None, step=0):
        f = np.ascontiguousarray(f, np.float64)
        us = None if ustar is None else np.ascontiguousarray(ustar, np.float64)
        self._chk(lib.tlvlbm_put_state(self.h, _ptr(f)[0], _ptr(us)[0], int(step)), "put_state")

    def links(self):
        L = self.stats()["cut_links"]
        node = np.zeros(L, np.int64)
        q = np.zeros(L, np.int32)
        eta = np.zeros(L)
        Nb = np.zeros((L, 3))
        bid = np.zeros(L, np.int32)
        self._chk(lib.tlvlbm_get_links(self.h, _ptr(node)[0], _ptr(q)[0], _ptr(eta)[0], _ptr(Nb)[0], _ptr(bid)[0]),
                  "get_links")
        return dict(node=node, q=q, eta=eta, N=Nb[:, : self.D], bid=bid)

    def stats(self):
        s = Stats()
        self._chk(lib.tlvlbm_stats(self.h, C.byref(s)), "stats")
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def synchronize(self):
        self._chk(lib.tlvlbm_synchronize(self.h), "synchronize")

    def population_bytes(self):
        return int(lib.tlvlbm_population_bytes(self.h))


def cut_links_noalloc(D, n, dx, phi, capacity, node, q, eta=None, Nb=None, bid_out=None, bid=None, origin=None,
                      periodic_mask=0, stream=None):
    """tlvlbm_cut_links_noalloc: the cut-link table of a level set with no
    device allocation.  phi [N] float64, bid [N] uint8 (or None), and the
    outputs node [cap] int64, q [cap] int32, eta [cap] float64, Nb [cap, 3]
    float64, bid_out [cap] int32 are contiguous device tensors owned by the
    caller (capacity = their length).  Returns the number of cut links; raises
    TlvlbmError (with .n_links set) when it exceeds the capacity."""
    g = Grid()
    for a in range(3):
        g.n[a] = int(n[a]) if a < D else 1
        g.origin[a] = (origin[a] if origin is not None and a < len(origin) else 0.0)
    g.dx = dx
    g.periodic_mask = periodic_mask
    nl = C.c_int64(0)
    st = lib.tlvlbm_cut_links_noalloc(C.byref(g), D, _ptr(phi)[0], _ptr(bid)[0], int(capacity), _ptr(node)[0],
                                      _ptr(q)[0], _ptr(eta)[0], _ptr(Nb)[0], _ptr(bid_out)[0], C.byref(nl), stream)
    if st:
        e = TlvlbmError(st, f"cut_links_noalloc (links: {nl.value}, capacity {capacity})")
        e.n_links = nl.value
        raise e
    return nl.value


def _handles(solvers):
    arr = (C.c_void_p * len(solvers))(*[s.h.value for s in solvers])
    return arr


def step_each(solvers, n):
    """Advance every solver n steps with per-instance launches (the reference
    for the batched path)."""
    st = lib.tlvlbm_step_each(_handles(solvers), len(solvers), int(n))
    if st:
        raise TlvlbmError(st, "step_each")


class Batch:
    """One tile-list launch per phase over many solvers (same lattice,
    precision and non-default stream; see include/tlvlbm.h)."""

    def __init__(self, solvers, use_graph=True):
        self.solvers = list(solvers)  # keep the contexts alive
        h = C.c_void_p()
        st = lib.tlvlbm_batch_create(_handles(self.solvers), len(self.solvers), C.byref(h))
        if st:
            raise TlvlbmError(st, "batch_create")
        self.h = h
        lib.tlvlbm_batch_set_graph(self.h, int(bool(use_graph)))

    def step(self, n=1):
        st = lib.tlvlbm_batch_step(self.h, int(n))
        if st:
            raise TlvlbmError(st, f"batch_step: {lib.tlvlbm_batch_last_error(self.h).decode()}")

    def autotune(self, reps=3):
        st = lib.tlvlbm_batch_autotune(self.h, int(reps))
        if st:
            raise TlvlbmError(st, f"batch_autotune: {lib.tlvlbm_batch_last_error(self.h).decode()}")
        return self.tiles()

    def set_tiles(self, tile_width, order):
        st = lib.tlvlbm_batch_set_tiles(self.h, int(tile_width), int(order))
        if st:
            raise TlvlbmError(st, f"batch_set_tiles: {lib.tlvlbm_batch_last_error(self.h).decode()}")

    def tiles(self):
        """(tile_width, order, {(order, width): mean ms per bulk launch})."""
        w, o = C.c_int32(0), C.c_int32(0)
        ms = (C.c_double * 6)()
        st = lib.tlvlbm_batch_get_tiles(self.h, C.byref(w), C.byref(o), ms)
        if st:
            raise TlvlbmError(st, "batch_get_tiles")
        return w.value, o.value, {(k // 3, (64, 128, 256)[k % 3]): ms[k] for k in range(6)}

    def close(self):
        if getattr(self, "h", None) and lib is not None:
            lib.tlvlbm_batch_destroy(self.h)
            self.h = None

    __del__ = close


_RUN_FN = None


def _run_fn():
    """torch.autograd.Function over tlvlbm_adjoint_record /
    tlvlbm_adjoint_backward (built on first use, so that importing the
    binding does not import torch)."""
    global _RUN_FN
    if _RUN_FN is not None:
        return _RUN_FN
    import torch

    def f64(t, dev):
        return t.detach().to(device=dev, dtype=torch.float64).contiguous()

    def ready(dev):
        # the library works on its own stream: torch's writes must be done
        if dev.type == "cuda":
            torch.cuda.current_stream(dev).synchronize()

    class _Run(torch.autograd.Function):
        @staticmethod
        def forward(ctx, mat, v0, dv0, solver, n, U0, dU0, segment, fibre):
            dev = v0.device
            D, M, N = solver.D, solver.M, solver.N
            mu, lam = (float(x) for x in mat.detach().to("cpu", torch.float64))
            U = f64(torch.as_tensor(U0), dev).clone()
            U[:D] = f64(v0, dev)
            if dU0 is None and dv0 is None:
                dU = None
            else:
                dU = f64(torch.as_tensor(dU0), dev).clone() if dU0 is not None else \
                    torch.zeros((D, M, N), dtype=torch.float64, device=dev)
                if dv0 is not None:
                    dU[:, :D] = f64(dv0, dev)
            ready(dev)
            solver.set_material(mu, lam, fibre)
            solver.set_state(U, dU0=dU)
            solver.adjoint_record(n, segment=segment)  # the forward, keeping its tape
            Uo = torch.empty((M, N), dtype=torch.float64, device=dev)
            uo = torch.empty((D, N), dtype=torch.float64, device=dev)
            solver.moments_into(U=Uo, u=uo)
            ctx.run = (solver, dU is not None and dv0 is not None)
            ctx.devices = (mat.device, dev)
            return Uo, uo

        @staticmethod
        def backward(ctx, gU, gu):
            solver, want_d = ctx.run
            dev = ctx.devices[1]
            D, M, N = solver.D, solver.M, solver.N
            gv = torch.empty((D, N), dtype=torch.float64, device=dev)
            gd = torch.empty((D, M, N), dtype=torch.float64, device=dev) if want_d else None
            gU = None if gU is None else f64(gU, dev)
            gu = None if gu is None else f64(gu, dev)
            ready(dev)
            gm, _, _, _ = solver.adjoint_backward(gU, gu, grad_v0=gv, grad_u0=False,
                                                  grad_dU0=gd if want_d else False)
            gmat = torch.tensor(gm, dtype=torch.float64, device=ctx.devices[0])
            gdv = gd[:, :D].contiguous() if want_d else None
            return gmat, gv, gdv, None, None, None, None, None, None

    _RUN_FN = _Run
    return _Run


def run_differentiable(solver, mat, v0, n, U0, dU0=None, segment=0, fibre=None, dv0=None):
    """Differentiable run of n steps for torch autograd.

    mat: tensor (mu, lambda) [2]; v0: tensor [D][nodes], the velocity rows of
    the initial state; U0: the initial state [M][nodes] (its F rows are used,
    its velocity rows replaced by v0); dU0: its gradients [D][M][nodes] as for
    set_state (or None); dv0: optional tensor [D][D][nodes], dv0[A][i] =
    d v0_i / d X_A, replacing the velocity rows of dU0 and receiving its own
    gradient (build it from v0 with differentiable torch operations, and
    autograd carries dL/d dv0 back to v0: the initial velocity and its
    gradient then stay consistent).  Returns (U, u) after n steps as float64
    tensors on v0's device.  The forward is tlvlbm_adjoint_record (the run,
    with its checkpoints and tape) and the backward tlvlbm_adjoint_backward:
    no second forward and no host copies (device tensors stay on the device).
    The solver's boundary conditions and level set stay as set by the caller;
    it must not be stepped between forward and backward.  Every step runs in
    the library's kernels; this is argument marshalling."""
    return _run_fn().apply(mat, v0, dv0, solver, int(n), U0, dU0, int(segment), fibre)
