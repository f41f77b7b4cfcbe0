"""ctypes binding of libctm.so (include/ctm.h).  Argument marshalling only.

Every computation happens inside the HIP library; this module converts numpy
arrays (or device pointers) to the C ABI and raises ``CtmError`` on a
non-zero status.  It never falls back to anything else: if the library is
missing, ``load()`` raises.
"""
import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libctm.so")

CTM_OK, CTM_EINVAL, CTM_ENOMEM, CTM_EDEVICE, CTM_ENUMERIC, CTM_ETOOBIG, CTM_EAGAIN, CTM_ECANCELED = \
    0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "CTM_OK", -1: "CTM_EINVAL", -2: "CTM_ENOMEM", -3: "CTM_EDEVICE", -4: "CTM_ENUMERIC",
                -5: "CTM_ETOOBIG", -6: "CTM_EAGAIN", -7: "CTM_ECANCELED"}
CTM_F64, CTM_F32, CTM_BF16, CTM_F16_SPLIT = 0, 1, 2, 3
PRECISIONS = {"f64": CTM_F64, "f32": CTM_F32, "bf16": CTM_BF16, "f16split": CTM_F16_SPLIT}
CTM_LEFT, CTM_RIGHT, CTM_UP, CTM_DOWN = 0, 1, 2, 3
DIRS = {"left": CTM_LEFT, "right": CTM_RIGHT, "up": CTM_UP, "down": CTM_DOWN}

# Every symbol include/ctm.h declares.
EXPORTS = (
    "ctm_init", "ctm_move", "ctm_sweep", "ctm_projectors", "ctm_enlarged_corner",
    "ctm_expect_1site", "ctm_expect_2site", "ctm_rho_1site", "ctm_rho_2site", "ctm_impurity",
    "ctm_log_kappa", "ctm_env_bytes", "ctm_get_env", "ctm_set_env", "ctm_move_count", "ctm_cut_stats",
    "ctm_footprint_bytes", "ctm_last_error", "ctm_free", "ctm_timing_enable", "ctm_timing_read",
    "ctm_queue_create", "ctm_queue_submit", "ctm_queue_poll", "ctm_queue_wait",
    "ctm_queue_cancel", "ctm_queue_destroy", "ctm_correlation", "ctm_transfer_spectrum",
    "ctm_xi_extrapolate", "ctm_expect_2site_noalloc",
    "ctm_su_create", "ctm_su_set_hamiltonians", "ctm_su_run", "ctm_su_stats", "ctm_su_get",
    "ctm_su_get_itps", "ctm_su_mfe", "ctm_su_mfe_energy", "ctm_su_last_error", "ctm_su_free",
    "ctm_fu_step", "ctm_get_tensors",
)


class ctm_su_config(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int), ("Ly", ctypes.c_int), ("d", ctypes.c_int), ("D", ctypes.c_int),
                ("batch", ctypes.c_int), ("stream", ctypes.c_void_p), ("complex_tensors", ctypes.c_int)]


class CtmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ctm_config(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int), ("Ly", ctypes.c_int), ("d", ctypes.c_int), ("D", ctypes.c_int),
                ("chi", ctypes.c_int), ("layers", ctypes.c_int), ("prec", ctypes.c_int),
                ("svd_rel_cutoff", ctypes.c_double), ("rsvd_oversample", ctypes.c_int),
                ("rsvd_power_iters", ctypes.c_int), ("seed", ctypes.c_uint64),
                ("stream", ctypes.c_void_p), ("projector_path", ctypes.c_int)]


CTM_PATH_AUTO, CTM_PATH_HOUSEHOLDER = 0, 1
PATHS = {"auto": CTM_PATH_AUTO, "householder": CTM_PATH_HOUSEHOLDER}


CTM_MAX_OBS, CTM_MAX_SITES = 8, 16


class ctm_request(ctypes.Structure):
    _fields_ = [("cfg", ctm_config), ("tensors", ctypes.POINTER(ctypes.c_double)),
                ("tensors_on_device", ctypes.c_int),
                ("bond_op", ctypes.POINTER(ctypes.c_double)),
                ("onsite_op", ctypes.POINTER(ctypes.c_double)),
                ("n_obs", ctypes.c_int), ("obs_ops", ctypes.POINTER(ctypes.c_double)),
                ("n_obs2", ctypes.c_int), ("obs2_ops", ctypes.POINTER(ctypes.c_double)),
                ("tol", ctypes.c_double), ("max_sweeps", ctypes.c_int), ("tag", ctypes.c_uint64)]


PHASES = ("contract_gemm", "sketch_gemm", "absorb", "factorise", "other")


class ctm_timing(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 5), ("ms", ctypes.c_double * 5), ("flops", ctypes.c_double * 5)]


class ctm_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("converged", ctypes.c_int), ("sweeps", ctypes.c_int),
                ("delta", ctypes.c_double), ("energy_per_site", ctypes.c_double),
                ("obs", (ctypes.c_double * CTM_MAX_SITES) * CTM_MAX_OBS),
                ("obs2", ((ctypes.c_double * 2) * CTM_MAX_SITES) * CTM_MAX_OBS),
                ("tag", ctypes.c_uint64),
                ("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64)]

    def observable(self, k, nsites):
        """<O_k> per site (one-site observable k of the request)."""
        return np.array([self.obs[k][i] for i in range(nsites)])

    def observable2(self, k, nsites):
        """<O2_k> per site and bond direction (+x, +y), shape (nsites, 2)."""
        return np.array([[self.obs2[k][i][dr] for dr in range(2)] for i in range(nsites)])


_lib = None
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)


def load(path=LIB_PATH):
    """Load libctm.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} not built; run paper_2112_13184_amd.build.build()")
    # PyTorch wheels bundle their own HIP runtime (same soname as the system
    # one).  Loading torch first makes the library bind to that runtime, so
    # that one runtime serves the process: device pointers and streams from
    # torch are then valid arguments of the library (and torch still finds
    # the device after the library has used it).
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    V, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    sig = {
        "ctm_init": (I, [ctypes.POINTER(ctm_config), _DP, I, _DP, ctypes.POINTER(V)]),
        "ctm_move": (I, [V, I]),
        "ctm_sweep": (I, [V, I, D, _IP, _DP, _IP]),
        "ctm_projectors": (I, [V, I, I, I, _DP, _DP, _IP]),
        "ctm_enlarged_corner": (I, [V, I, I, _DP]),
        "ctm_expect_1site": (I, [V, I, _DP, _DP]),
        "ctm_expect_2site": (I, [V, I, I, _DP, _DP]),
        "ctm_rho_1site": (I, [V, I, _DP]),
        "ctm_rho_2site": (I, [V, I, I, _DP]),
        "ctm_impurity": (I, [V, I, _DP, _DP]),
        "ctm_log_kappa": (I, [V, _DP]),
        "ctm_env_bytes": (S, [V]),
        "ctm_get_env": (I, [V, I, _DP, S, _IP]),
        "ctm_set_env": (I, [V, I, _DP, S, _IP]),
        "ctm_move_count": (I, [V, ctypes.POINTER(ctypes.c_int64)]),
        "ctm_cut_stats": (I, [V, ctypes.POINTER(ctypes.c_int64)]),
        "ctm_footprint_bytes": (S, [ctypes.POINTER(ctm_config)]),
        "ctm_last_error": (ctypes.c_char_p, [V]),
        "ctm_free": (None, [V]),
        "ctm_timing_enable": (I, [V, I]),
        "ctm_timing_read": (I, [V, ctypes.POINTER(ctm_timing)]),
        "ctm_queue_create": (I, [S, I, V, ctypes.POINTER(V)]),
        "ctm_queue_submit": (I, [V, ctypes.POINTER(ctm_request), ctypes.POINTER(ctypes.c_uint64)]),
        "ctm_queue_poll": (I, [V, ctypes.c_uint64, ctypes.POINTER(ctm_result)]),
        "ctm_queue_wait": (I, [V, ctypes.c_uint64, I, ctypes.POINTER(ctm_result)]),
        "ctm_queue_cancel": (I, [V, ctypes.c_uint64]),
        "ctm_queue_destroy": (None, [V]),
        "ctm_correlation": (I, [V, I, I, _DP, _DP, I, _DP]),
        "ctm_transfer_spectrum": (I, [V, I, I, I, _DP, _DP, _DP, _DP]),
        "ctm_xi_extrapolate": (I, [I, _DP, _DP, _DP, _DP]),
        "ctm_expect_2site_noalloc": (I, [V, I, I, _DP, _DP]),
        "ctm_su_create": (I, [ctypes.POINTER(ctm_su_config), _DP, _DP, ctypes.POINTER(V)]),
        "ctm_su_set_hamiltonians": (I, [V, _DP, _DP]),
        "ctm_su_run": (I, [V, I]),
        "ctm_su_stats": (I, [V, _DP, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_long)]),
        "ctm_su_get": (I, [V, _DP, _DP]),
        "ctm_su_get_itps": (I, [V, _DP, I]),
        "ctm_su_mfe": (I, [V, _DP, _DP]),
        "ctm_su_mfe_energy": (I, [V, _DP, _DP, _DP]),
        "ctm_su_last_error": (ctypes.c_char_p, [V]),
        "ctm_su_free": (None, [V]),
        "ctm_fu_step": (I, [V, _DP, D, I, I]),
        "ctm_get_tensors": (I, [V, _DP]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(_DP)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_config(Lx, Ly, D, chi, d=2, layers=2, prec="f64", svd_rel_cutoff=0.0, rsvd_oversample=32,
                rsvd_power_iters=1, seed=0, stream=None, projector_path="auto"):
    cfg = ctm_config()
    cfg.Lx, cfg.Ly, cfg.d, cfg.D, cfg.chi, cfg.layers = Lx, Ly, d, D, chi, layers
    cfg.prec = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    cfg.svd_rel_cutoff = svd_rel_cutoff
    cfg.rsvd_oversample, cfg.rsvd_power_iters = rsvd_oversample, rsvd_power_iters
    cfg.seed = seed
    cfg.stream = stream
    cfg.projector_path = PATHS[projector_path] if isinstance(projector_path, str) else int(projector_path)
    return cfg


def ctm_footprint_bytes(cfg):
    return int(load().ctm_footprint_bytes(ctypes.byref(cfg)))


def ctm_xi_extrapolate(e1, e2):
    """Eq. (9) over runs at several chi: (1/xi(inf), k)."""
    a, b = _f64(e1), _f64(e2)
    inv, k = ctypes.c_double(), ctypes.c_double()
    st = load().ctm_xi_extrapolate(len(a), _dp(a), _dp(b), ctypes.byref(inv), ctypes.byref(k))
    if st != CTM_OK:
        raise CtmError(st, "ctm_xi_extrapolate")
    return inv.value, k.value


class Ctm:
    """One CTMRG context (ctm_ctx) on the GPU."""

    def __init__(self, tensors, Lx, Ly, D, chi, d=2, layers=2, boundary=None, device_ptr=None, **kw):
        lib = load()
        self.cfg = make_config(Lx, Ly, D, chi, d=d if layers == 2 else 1, layers=layers, **kw)
        self.Lx, self.Ly, self.D, self.chi, self.layers = Lx, Ly, D, chi, layers
        self.d = d if layers == 2 else 1
        self.Db = D * D if layers == 2 else D
        self.n = chi * self.Db
        h = ctypes.c_void_p()
        if device_ptr is not None:
            tp, on_dev = ctypes.cast(ctypes.c_void_p(int(device_ptr)), _DP), 1
            self._keep = None
        else:
            arr = _f64(np.concatenate([np.asarray(t, dtype=np.float64).reshape(-1) for t in tensors]))
            tp, on_dev = _dp(arr), 0
            self._keep = arr
        b = None
        if boundary is not None:
            self._bnd = _f64(boundary).reshape(-1)
            b = _dp(self._bnd)
        st = lib.ctm_init(ctypes.byref(self.cfg), tp, on_dev, b, ctypes.byref(h))
        if st != CTM_OK:
            raise CtmError(st, lib.ctm_last_error(None).decode())
        self._h = h
        self._lib = lib

    def _check(self, st):
        if st != CTM_OK:
            raise CtmError(st, self._lib.ctm_last_error(self._h).decode())

    def ctm_move(self, direction):
        d = DIRS[direction] if isinstance(direction, str) else int(direction)
        self._check(self._lib.ctm_move(self._h, d))

    def ctm_sweep(self, max_sweeps, tol):
        done, conv, delta = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        self._check(self._lib.ctm_sweep(self._h, max_sweeps, tol, ctypes.byref(done),
                                        ctypes.byref(delta), ctypes.byref(conv)))
        return done.value, delta.value, bool(conv.value)

    def ctm_projectors(self, direction, x, y):
        d = DIRS[direction] if isinstance(direction, str) else int(direction)
        P = np.zeros((self.chi, self.n))
        Pt = np.zeros((self.n, self.chi))
        k = ctypes.c_int()
        self._check(self._lib.ctm_projectors(self._h, d, x, y, _dp(P), _dp(Pt), ctypes.byref(k)))
        return P, Pt, k.value

    def ctm_enlarged_corner(self, corner, site):
        E = np.zeros((self.n, self.n))
        self._check(self._lib.ctm_enlarged_corner(self._h, corner, site, _dp(E)))
        return E

    def ctm_expect_1site(self, site, op):
        v = ctypes.c_double()
        o = _f64(op)
        self._check(self._lib.ctm_expect_1site(self._h, site, _dp(o), ctypes.byref(v)))
        return v.value

    def ctm_expect_2site(self, site, direction, op):
        v = ctypes.c_double()
        o = _f64(op)
        self._check(self._lib.ctm_expect_2site(self._h, site, direction, _dp(o), ctypes.byref(v)))
        return v.value

    def ctm_expect_2site_noalloc(self, site, direction, op):
        """ctm_expect_2site with its transients in the library's fixed
        device array (no device allocation in the call)."""
        v = ctypes.c_double()
        o = _f64(op)
        self._check(self._lib.ctm_expect_2site_noalloc(self._h, site, direction, _dp(o), ctypes.byref(v)))
        return v.value

    def ctm_rho_1site(self, site):
        r = np.zeros((self.d, self.d))
        self._check(self._lib.ctm_rho_1site(self._h, site, _dp(r)))
        return r

    def ctm_rho_2site(self, site, direction):
        r = np.zeros((self.d * self.d, self.d * self.d))
        self._check(self._lib.ctm_rho_2site(self._h, site, direction, _dp(r)))
        return r

    def ctm_correlation(self, site, direction, opA, opB, rmax):
        """C(r) = <A(site) B(site + r e)>, r = 0..rmax, e = +x (0) or +y (1)."""
        out = np.zeros(rmax + 1)
        a, b = _f64(opA), _f64(opB)
        self._check(self._lib.ctm_correlation(self._h, site, direction, _dp(a), _dp(b), rmax, _dp(out)))
        return out

    def ctm_transfer_spectrum(self, direction, line, nev):
        """(eigenvalues (complex, by modulus), e_k (k = 1..nev-1), xi)."""
        re, im, e = np.zeros(nev), np.zeros(nev), np.zeros(max(nev - 1, 1))
        xi = ctypes.c_double()
        self._check(self._lib.ctm_transfer_spectrum(self._h, direction, line, nev, _dp(re), _dp(im), _dp(e),
                                                    ctypes.byref(xi)))
        return re + 1j * im, e[:nev - 1], xi.value

    def ctm_impurity(self, site, b):
        v = ctypes.c_double()
        bb = _f64(b)
        self._check(self._lib.ctm_impurity(self._h, site, _dp(bb), ctypes.byref(v)))
        return v.value

    def ctm_fu_step(self, H, tau, als_iters=5, env_sweeps=1):
        """One full-update Trotter step; H [N][2][d^2][d^2]."""
        h = _f64(np.asarray(H, dtype=np.float64)).reshape(-1)
        self._check(self._lib.ctm_fu_step(self._h, _dp(h), float(tau), int(als_iters), int(env_sweeps)))

    def ctm_get_tensors(self):
        out = np.empty((self.Lx * self.Ly,) + (self.D,) * 4 + (self.d,))
        self._check(self._lib.ctm_get_tensors(self._h, _dp(out)))
        return out

    def ctm_log_kappa(self):
        v = ctypes.c_double()
        self._check(self._lib.ctm_log_kappa(self._h, ctypes.byref(v)))
        return v.value

    def ctm_get_env(self, site):
        nb = int(self._lib.ctm_env_bytes(self._h))
        buf = np.zeros(nb // 8)
        dims = np.zeros(16, dtype=np.int32)
        self._check(self._lib.ctm_get_env(self._h, site, _dp(buf), nb,
                                          dims.ctypes.data_as(_IP)))
        cc, tt = self.chi * self.chi, self.chi * self.chi * self.Db
        C = [buf[k * cc:(k + 1) * cc].reshape(self.chi, self.chi) for k in range(4)]
        T = [buf[4 * cc + k * tt:4 * cc + (k + 1) * tt].reshape(self.chi, self.chi, self.Db)
             for k in range(4)]
        return C, T, dims.reshape(2, 4, 2)

    def ctm_set_env(self, site, C, T, dims=None):
        buf = _f64(np.concatenate([np.asarray(x).reshape(-1) for x in list(C) + list(T)]))
        dp = None
        if dims is not None:
            self._dims = np.ascontiguousarray(np.asarray(dims).reshape(16), dtype=np.int32)
            dp = self._dims.ctypes.data_as(_IP)
        self._check(self._lib.ctm_set_env(self._h, site, _dp(buf), buf.nbytes, dp))

    def ctm_move_count(self):
        m = ctypes.c_int64()
        self._check(self._lib.ctm_move_count(self._h, ctypes.byref(m)))
        return m.value

    def ctm_cut_stats(self):
        """(identity, batched randomized SVD, fallback) cut counts since init."""
        c = (ctypes.c_int64 * 3)()
        self._check(self._lib.ctm_cut_stats(self._h, c))
        return tuple(int(v) for v in c)

    def ctm_timing_enable(self, on=True):
        """on: False (off), True or 1 (every phase), 2 (the sketch GEMMs only)."""
        self._check(self._lib.ctm_timing_enable(self._h, int(on)))

    def ctm_timing_read(self):
        t = ctm_timing()
        self._check(self._lib.ctm_timing_read(self._h, ctypes.byref(t)))
        return {name: dict(launches=int(t.launches[i]), ms=float(t.ms[i]), flops=float(t.flops[i]))
                for i, name in enumerate(PHASES)}

    def ctm_free(self):
        if getattr(self, "_h", None):
            self._lib.ctm_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.ctm_free()
        except Exception:
            pass


class Queue:
    """A ctm_queue: CTMRG solves admitted by HBM footprint and run concurrently."""

    def __init__(self, hbm_budget_bytes, max_active, stream=None):
        lib = load()
        q = ctypes.c_void_p()
        st = lib.ctm_queue_create(int(hbm_budget_bytes), int(max_active), stream, ctypes.byref(q))
        if st != CTM_OK:
            raise CtmError(st, "ctm_queue_create failed")
        self._lib, self._q = lib, q

    def submit(self, tensors, Lx, Ly, D, chi, bond_op, onsite_op=None, tol=1e-10, max_sweeps=40, tag=0,
               d=2, obs=(), obs2=(), device_ptr=None, **kw):
        """Returns (status, ticket); inputs are copied by the library.  obs /
        obs2: one-site (d x d) and two-site (d^2 x d^2) observables to measure;
        device_ptr: address of the site tensors in device memory (then
        ``tensors`` is ignored)."""
        req = ctm_request()
        req.cfg = make_config(Lx, Ly, D, chi, d=d, **kw)
        keep = []
        if device_ptr is not None:
            req.tensors = ctypes.cast(ctypes.c_void_p(int(device_ptr)), _DP)
            req.tensors_on_device = 1
        else:
            t = _f64(np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1) for a in tensors]))
            keep.append(t)
            req.tensors = _dp(t)
        b = _f64(bond_op)
        keep.append(b)
        req.bond_op = _dp(b)
        if onsite_op is not None:
            o = _f64(onsite_op)
            keep.append(o)
            req.onsite_op = _dp(o)
        if len(obs):
            a = _f64(np.stack([np.asarray(x, dtype=np.float64) for x in obs]))
            keep.append(a)
            req.n_obs, req.obs_ops = len(obs), _dp(a)
        if len(obs2):
            a = _f64(np.stack([np.asarray(x, dtype=np.float64) for x in obs2]))
            keep.append(a)
            req.n_obs2, req.obs2_ops = len(obs2), _dp(a)
        req.tol, req.max_sweeps, req.tag = float(tol), int(max_sweeps), int(tag)
        ticket = ctypes.c_uint64()
        st = self._lib.ctm_queue_submit(self._q, ctypes.byref(req), ctypes.byref(ticket))
        return st, ticket.value

    def poll(self, ticket):
        r = ctm_result()
        st = self._lib.ctm_queue_poll(self._q, ticket, ctypes.byref(r))
        return st, r

    def wait(self, ticket, timeout_ms=-1):
        r = ctm_result()
        st = self._lib.ctm_queue_wait(self._q, ticket, int(timeout_ms), ctypes.byref(r))
        return st, r

    def cancel(self, ticket):
        return self._lib.ctm_queue_cancel(self._q, ticket)

    def destroy(self):
        if self._q:
            self._lib.ctm_queue_destroy(self._q)
            self._q = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class SimpleUpdate:
    """A ctm_su handle: simple-update imaginary-time evolution of `batch`
    independent problems, and their mean-field-environment density matrices.

    gamma: [batch][N][D, D, D, D, d] (or a list of per-problem lists of site
    tensors), lam: [batch][N][2][D] bond weights (see include/ctm.h).  With
    complex_tensors the tensors, Hamiltonians and density matrices are
    complex128 arrays (passed to the library as (re, im) pairs)."""

    def __init__(self, gamma, lam, Lx, Ly, D, d=2, batch=None, stream=None, complex_tensors=False):
        lib = load()
        self.cplx = bool(complex_tensors)
        g = self._scal(gamma)
        lm = _f64(np.asarray(lam, dtype=np.float64)).reshape(-1)
        N = Lx * Ly
        w = 2 if self.cplx else 1
        if batch is None:
            batch = g.size // (N * D ** 4 * d * w)
        if g.size != batch * N * D ** 4 * d * w or lm.size != batch * N * 2 * D:
            raise CtmError(CTM_EINVAL, "gamma / lambda sizes do not match the shape")
        cfg = ctm_su_config(Lx, Ly, d, D, int(batch), stream, 1 if self.cplx else 0)
        h = ctypes.c_void_p()
        st = lib.ctm_su_create(ctypes.byref(cfg), _dp(g), _dp(lm), ctypes.byref(h))
        if st != CTM_OK:
            raise CtmError(st, (lib.ctm_su_last_error(None) or b"").decode())
        self._lib, self._h = lib, h
        self.Lx, self.Ly, self.D, self.d, self.batch, self.N = Lx, Ly, D, d, int(batch), N

    def _scal(self, x):
        """Flat FP64 buffer of a tensor argument ((re, im) pairs when complex)."""
        if self.cplx:
            return np.ascontiguousarray(np.asarray(x, dtype=np.complex128)).reshape(-1).view(np.float64)
        return _f64(np.asarray(x, dtype=np.float64)).reshape(-1)

    def _out(self, shape):
        return np.empty(shape, dtype=np.complex128 if self.cplx else np.float64)

    def _ptr(self, a):
        return a.reshape(-1).view(np.float64).ctypes.data_as(_DP) if self.cplx else _dp(a)

    def _check(self, st):
        if st != CTM_OK:
            raise CtmError(st, (self._lib.ctm_su_last_error(self._h) or b"").decode())

    def set_hamiltonians(self, H, tau):
        """H: [batch][N][2][d^2][d^2]; tau: scalar or [batch]."""
        Hh = self._scal(H)
        t = _f64(np.broadcast_to(np.asarray(tau, dtype=np.float64), (self.batch,)))
        if Hh.size != self.batch * self.N * 2 * self.d ** 4 * (2 if self.cplx else 1):
            raise CtmError(CTM_EINVAL, "H size does not match the shape")
        self._check(self._lib.ctm_su_set_hamiltonians(self._h, _dp(Hh), _dp(t)))

    def run(self, nsteps):
        self._check(self._lib.ctm_su_run(self._h, int(nsteps)))

    def stats(self):
        ms, la, bu = ctypes.c_double(), ctypes.c_long(), ctypes.c_long()
        self._check(self._lib.ctm_su_stats(self._h, ctypes.byref(ms), ctypes.byref(la), ctypes.byref(bu)))
        return ms.value, la.value, bu.value

    def get(self):
        """(gamma [batch, N, D, D, D, D, d], lam [batch, N, 2, D])."""
        g = self._out((self.batch, self.N) + (self.D,) * 4 + (self.d,))
        lm = np.empty((self.batch, self.N, 2, self.D))
        self._check(self._lib.ctm_su_get(self._h, self._ptr(g), _dp(lm)))
        return g, lm

    def get_itps(self, device_ptr=None):
        """A_s = G_s sqrt(weights): a host array [batch, N, D, D, D, D, d], or
        written to device memory at device_ptr."""
        if device_ptr is not None:
            self._check(self._lib.ctm_su_get_itps(self._h, ctypes.cast(ctypes.c_void_p(int(device_ptr)), _DP), 1))
            return None
        a = self._out((self.batch, self.N) + (self.D,) * 4 + (self.d,))
        self._check(self._lib.ctm_su_get_itps(self._h, self._ptr(a), 0))
        return a

    def mfe(self):
        """(rho1 [batch, N, d, d], rho2 [batch, N, 2, d^2, d^2]), unit trace."""
        r1 = self._out((self.batch, self.N, self.d, self.d))
        r2 = self._out((self.batch, self.N, 2, self.d ** 2, self.d ** 2))
        self._check(self._lib.ctm_su_mfe(self._h, self._ptr(r1), self._ptr(r2)))
        return r1, r2

    def mfe_energy(self, onsite=None):
        """(energy per site [batch], bond energies [batch, N, 2])."""
        e = np.empty(self.batch)
        be = np.empty((self.batch, self.N, 2))
        o = None
        if onsite is not None:
            o = self._scal(np.broadcast_to(np.asarray(onsite), (self.batch, self.d, self.d)))
        self._check(self._lib.ctm_su_mfe_energy(self._h, _dp(o) if o is not None else None, _dp(e), _dp(be)))
        return e, be

    def free(self):
        if getattr(self, "_h", None):
            self._lib.ctm_su_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
