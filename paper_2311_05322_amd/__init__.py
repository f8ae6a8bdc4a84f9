"""Python binding of libmx.so, the MI355X (gfx950) Maxwell/Schwarz solver.

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Arrays may be numpy arrays (host) or torch tensors on the GPU
(device pointers are passed straight through).  The C ABI is declared in
include/mx.h; the names here mirror it.  A process that uses torch on the GPU
as well imports torch before the first call into the library: torch ships
its own HIP runtime under the same soname, the first one loaded serves both,
and torch finds no device when it is not its own.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmx.so")

MX_OK, MX_EINVAL, MX_ENOMEM, MX_ESTATE, MX_ENOTCONV, MX_EPIVOT, MX_EHIP = 0, -1, -2, -3, -4, -5, -6
MX_EPS_P0, MX_EPS_P1 = 0, 1
MX_PREC_C128, MX_PREC_C64 = 0, 1
MX_KRYLOV_PSEUDO_BLOCK, MX_KRYLOV_BLOCK, MX_KRYLOV_BLOCK_CGS2 = 0, 1, 2

EXPORTS = ["mx_create", "mx_destroy", "mx_assemble", "mx_setup_schwarz", "mx_solve", "mx_solve_rhs",
           "mx_apply_operator", "mx_apply_preconditioner", "mx_apply_preconditioner_noalloc", "mx_get_sizes", "mx_get_topology",
           "mx_get_matrix_values", "mx_get_partition", "mx_get_local_matrix", "mx_point_functionals",
           "mx_set_stream", "mx_set_autotune", "mx_set_lu_group", "mx_set_tuning", "mx_get_tuning", "mx_set_graphs", "mx_set_profiling", "mx_get_kernel_times", "mx_gradient", "mx_coarse_num_params", "mx_coarse_init",
           "mx_coarse_set_weights", "mx_coarse_get_weights", "mx_coarse_features", "mx_coarse_forward",
           "mx_coarse_loss_grad", "mx_coarse_hidden", "mx_coarse_adam_step", "mx_coarse_collect", "mx_coarse_clear", "mx_coarse_train", "mx_set_ports",
           "mx_solve_ports", "mx_set_krylov", "mx_last_error"]

KERNEL_CLASSES = ["lu_panel", "lu_rowpanel", "lu_update", "lu_inv", "trsm_lower", "trsm_upper", "spmm",
                  "restrict", "prolong", "cgs", "assemble", "local", "coarse"]


class MxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class c128(ct.Structure):
    _fields_ = [("re", ct.c_double), ("im", ct.c_double)]


class Mesh(ct.Structure):
    _fields_ = [("nv", ct.c_int32), ("nt", ct.c_int32), ("xyz", ct.c_void_p), ("tet", ct.c_void_p)]


class SchwarzOpts(ct.Structure):
    _fields_ = [("precision", ct.c_int32), ("restart", ct.c_int32), ("maxit", ct.c_int32), ("factor", ct.c_int32),
                ("coarse", ct.c_int32)]


class Sources(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("pos", ct.c_void_p), ("moment", ct.c_void_p)]


class Port(ct.Structure):
    """Waveguide port: rectangle (centre, outward normal, broad side u, a x b)
    filled with relative permittivity eps; TE10 incidence (Sec. IV-B)."""
    _fields_ = [("centre", ct.c_double * 3), ("normal", ct.c_double * 3), ("u", ct.c_double * 3),
                ("a", ct.c_double), ("b", ct.c_double), ("eps", c128)]


class SolveInfo(ct.Structure):
    _fields_ = [("iters", ct.c_void_p), ("relres", ct.c_void_p), ("iters_max", ct.c_int32),
                ("cycles", ct.c_int32), ("t_iter", ct.c_double), ("fallback", ct.c_int32),
                ("t_assemble", ct.c_double), ("t_setup", ct.c_double), ("t_lu", ct.c_double)]


def _info_dict(info, iters, relres, rc):
    return {"iters": iters, "relres": relres, "iters_max": info.iters_max, "cycles": info.cycles,
            "t_iter": info.t_iter, "converged": rc == MX_OK, "fallback": info.fallback,
            "t_assemble": info.t_assemble, "t_setup": info.t_setup, "t_lu": info.t_lu}


class Sizes(ct.Structure):
    _fields_ = [("nv", ct.c_int64), ("nt", ct.c_int64), ("ne", ct.c_int64), ("nnz", ct.c_int64),
                ("nbface", ct.c_int64), ("nsub", ct.c_int32), ("overlap", ct.c_int32), ("ncolour", ct.c_int32),
                ("sum_ni", ct.c_int64), ("sum_Ni2", ct.c_int64), ("nb", ct.c_int32), ("lu_tiles", ct.c_int64),
                ("trsm_tiles_lower", ct.c_int64), ("trsm_tiles_upper", ct.c_int64)]


class Tuning(ct.Structure):
    _fields_ = [("spmm_variant", ct.c_int32), ("trsm_paired", ct.c_int32), ("trsm_cols", ct.c_int32),
                ("spmm_ms", ct.c_double * 3), ("trsm_ms", ct.c_double * 4), ("lu_group", ct.c_int32),
                ("lu_ms", ct.c_double * 4), ("from_cache", ct.c_int32)]


class KernelTimes(ct.Structure):
    _fields_ = [("ms", ct.c_double * 16), ("launches", ct.c_int64 * 16)]


_lib = None


def lib():
    """Load libmx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2311_05322_amd.build`")
        L = ct.CDLL(LIB_PATH)
        vp, i32, dbl = ct.c_void_p, ct.c_int32, ct.c_double
        sig = {
            "mx_create": [ct.POINTER(vp), ct.c_int, vp],
            "mx_destroy": [vp],
            "mx_assemble": [vp, ct.POINTER(Mesh), vp, ct.c_int, dbl, c128],
            "mx_setup_schwarz": [vp, i32, i32, ct.POINTER(SchwarzOpts)],
            "mx_solve": [vp, ct.POINTER(Sources), ct.POINTER(Sources), dbl, vp, vp, ct.POINTER(SolveInfo)],
            "mx_solve_rhs": [vp, vp, i32, dbl, vp, ct.POINTER(SolveInfo)],
            "mx_apply_operator": [vp, vp, vp, i32],
            "mx_apply_preconditioner": [vp, vp, vp, i32],
            "mx_apply_preconditioner_noalloc": [vp, vp, vp, i32],
            "mx_get_sizes": [vp, ct.POINTER(Sizes)],
            "mx_get_topology": [vp, vp, vp, vp, vp],
            "mx_get_matrix_values": [vp, vp],
            "mx_get_partition": [vp, vp, vp, vp, vp, vp],
            "mx_get_local_matrix": [vp, i32, vp],
            "mx_point_functionals": [vp, ct.POINTER(Sources), vp],
            "mx_set_stream": [vp, vp],
            "mx_set_profiling": [vp, ct.c_int],
            "mx_set_graphs": [vp, ct.c_int],
            "mx_set_autotune": [vp, ct.c_int],
            "mx_set_lu_group": [vp, i32],
            "mx_set_tuning": [vp, i32, i32, i32],
            "mx_get_tuning": [vp, vp],
            "mx_get_kernel_times": [vp, ct.POINTER(KernelTimes)],
            "mx_gradient": [vp, vp, vp, dbl, vp, ct.POINTER(dbl), ct.POINTER(SolveInfo)],
            "mx_coarse_init": [vp, ct.c_uint64],
            "mx_coarse_set_weights": [vp, vp, ct.c_int64, dbl, dbl],
            "mx_coarse_get_weights": [vp, vp, ct.c_int64, ct.POINTER(dbl), ct.POINTER(dbl)],
            "mx_coarse_features": [vp, vp, i32, vp],
            "mx_coarse_forward": [vp, vp, i32, vp],
            "mx_coarse_loss_grad": [vp, vp, vp, i32, ct.POINTER(dbl), vp],
            "mx_coarse_hidden": [vp, vp, i32, vp, vp],
            "mx_coarse_adam_step": [vp, vp, ct.c_int64, dbl],
            "mx_coarse_collect": [vp, ct.POINTER(Sources), i32, i32, dbl, ct.POINTER(i32)],
            "mx_coarse_clear": [vp],
            "mx_coarse_train": [vp, i32, i32, dbl, ct.c_uint64, vp],
            "mx_set_ports": [vp, i32, ct.POINTER(Port), i32],
            "mx_solve_ports": [vp, dbl, vp, vp, ct.POINTER(SolveInfo)],
            "mx_set_krylov": [vp, i32],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ct.c_int
        L.mx_coarse_num_params.argtypes = []
        L.mx_coarse_num_params.restype = ct.c_int64
        L.mx_last_error.argtypes = []
        L.mx_last_error.restype = ct.c_char_p
        _lib = L
    return _lib


def _check(rc, allow=()):
    if rc != MX_OK and rc not in allow:
        raise MxError(rc, lib().mx_last_error().decode())
    return rc


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a):
    """Raw pointer of a contiguous numpy array or torch tensor (host or device)."""
    if a is None:
        return None
    if _is_torch(a):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ct.c_void_p(a.data_ptr())
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError("array must be C-contiguous")
    return ct.c_void_p(a.ctypes.data)


def _sources(pos, mom):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mom = np.ascontiguousarray(mom, dtype=np.complex128)
    s = Sources(pos.shape[0], pos.ctypes.data, mom.ctypes.data)
    return s, (pos, mom)


class Context:
    """One solver context on one GPU (wraps mx_create / mx_destroy)."""

    def __init__(self, device: int = 0, stream=None):
        """stream: integer HIP stream handle (e.g. torch's Stream.cuda_stream)
        the context runs on; None gives it a stream of its own."""
        h = ct.c_void_p()
        _check(lib().mx_create(ct.byref(h), device, ct.c_void_p(stream) if stream else None))
        self._h = h
        self.nports = 0
        self.ne = 0

    def close(self):
        if getattr(self, "_h", None):
            lib().mx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_stream(self, stream):
        """Run on a caller HIP stream (integer handle, e.g. torch's
        Stream.cuda_stream); None returns to the context's own stream."""
        _check(lib().mx_set_stream(self._h, ct.c_void_p(stream) if stream else None))

    def set_profiling(self, enable=True):
        _check(lib().mx_set_profiling(self._h, 1 if enable else 0))

    def set_autotune(self, enable=True):
        _check(lib().mx_set_autotune(self._h, 1 if enable else 0))

    def set_tuning(self, spmm_variant=1, trsm_paired=1, trsm_cols=32):
        """Fix the kernel variants (the autotuner is switched off)."""
        _check(lib().mx_set_tuning(self._h, int(spmm_variant), int(trsm_paired), int(trsm_cols)))

    def set_lu_group(self, group=0):
        """Fix the factorisation's panels per trailing-update pass (1..16), or
        0 to let the autotuner pick it; takes effect at the next set-up."""
        _check(lib().mx_set_lu_group(self._h, int(group)))

    def tuning(self):
        """Variants picked by the autotuner and their measured times (ms)."""
        t = Tuning()
        _check(lib().mx_get_tuning(self._h, ct.byref(t)))
        return {"spmm_variant": t.spmm_variant, "trsm_paired": t.trsm_paired, "trsm_cols": t.trsm_cols,
                "spmm_ms": list(t.spmm_ms),
                "trsm_ms_first32_paired32_first16_paired16": list(t.trsm_ms),
                "lu_group": t.lu_group, "lu_ms_groups_1_2_4_8": list(t.lu_ms),
                "from_cache": {"solve": bool(t.from_cache & 1), "lu": bool(t.from_cache & 2)}}

    def set_krylov(self, block=True, two_pass=False):
        """Block FGMRES (one Krylov space for all right-hand sides; two_pass:
        block Gram-Schmidt and Cholesky QR applied twice) or the default
        pseudo-block FGMRES (one per right-hand side). With the learned term
        set up, block mode runs the judged learned steps first and continues
        with block FGMRES once the term is switched off."""
        mode = (MX_KRYLOV_BLOCK_CGS2 if two_pass else MX_KRYLOV_BLOCK) if block else MX_KRYLOV_PSEUDO_BLOCK
        _check(lib().mx_set_krylov(self._h, mode))

    def set_graphs(self, enable=True):
        """Replay captured HIP graphs for plain Arnoldi steps (default on)."""
        _check(lib().mx_set_graphs(self._h, 1 if enable else 0))

    def kernel_times(self):
        """{class: (milliseconds, launches)} since profiling was enabled."""
        k = KernelTimes()
        _check(lib().mx_get_kernel_times(self._h, ct.byref(k)))
        return {name: (k.ms[i], int(k.launches[i])) for i, name in enumerate(KERNEL_CLASSES)}

    # -- operator ------------------------------------------------------------
    def assemble(self, xyz, tet, eps, eps_kind, freq, eps_b, reuse_mesh=False):
        keep = []
        if reuse_mesh:
            mp = None
        else:
            xyz = np.ascontiguousarray(xyz, dtype=np.float64)
            tet = np.ascontiguousarray(tet, dtype=np.int32)
            keep += [xyz, tet]
            m = Mesh(xyz.shape[0], tet.shape[0], xyz.ctypes.data, tet.ctypes.data)
            mp = ct.byref(m)
        if not _is_torch(eps):
            eps = np.ascontiguousarray(eps, dtype=np.complex128)
        eb = complex(eps_b)
        _check(lib().mx_assemble(self._h, mp, _ptr(eps), int(eps_kind), float(freq), c128(eb.real, eb.imag)))
        self.ne = self.sizes().ne
        if not reuse_mesh:
            self.nports = 0  # a new mesh clears the ports
        del keep

    def setup_schwarz(self, nsub, overlap, precision=MX_PREC_C128, restart=15, maxit=2000, factor=True,
                      coarse=False):
        o = SchwarzOpts(int(precision), int(restart), int(maxit), 1 if factor else 0, 1 if coarse else 0)
        _check(lib().mx_setup_schwarz(self._h, int(nsub), int(overlap), ct.byref(o)))

    # -- solves ----------------------------------------------------------------
    def solve(self, pos, mom, rx=None, rtol=1e-8, E=None, S=None, want_E=True):
        """All-transmitter solve.  E/S may be preallocated host arrays or device
        tensors ([ne][ntx], [nrx][ntx] complex128); returns (E, S, info)."""
        tx, keep = _sources(pos, mom)
        rxs = None
        if rx is not None:
            rxs, keep2 = _sources(*rx)
            keep = keep + keep2
        ntx = tx.n
        nrx = rxs.n if rxs is not None else ntx
        if E is None and want_E:
            E = np.zeros((self.ne, ntx), dtype=np.complex128)
        if S is None:
            S = np.zeros((nrx, ntx), dtype=np.complex128)
        iters = np.zeros(ntx, dtype=np.int32)
        relres = np.zeros(ntx, dtype=np.float64)
        info = SolveInfo(iters.ctypes.data, relres.ctypes.data)
        rc = lib().mx_solve(self._h, ct.byref(tx), ct.byref(rxs) if rxs is not None else None, float(rtol),
                            _ptr(E), _ptr(S), ct.byref(info))
        _check(rc, allow=(MX_ENOTCONV,))
        return E, S, _info_dict(info, iters, relres, rc)

    def set_ports(self, ports, pec=True):
        """Waveguide ports (objects with centre, normal, u, a, b, eps) and, with
        pec, metallic walls on the rest of the boundary; [] restores the
        impedance boundary. Re-assembles the operator: set up Schwarz after."""
        arr = (Port * max(1, len(ports)))()
        for i, p in enumerate(ports):
            e = complex(p.eps)
            arr[i] = Port((ct.c_double * 3)(*p.centre), (ct.c_double * 3)(*p.normal), (ct.c_double * 3)(*p.u),
                          float(p.a), float(p.b), c128(e.real, e.imag))
        _check(lib().mx_set_ports(self._h, len(ports), arr, 1 if pec else 0))
        self.nports = len(ports)

    def solve_ports(self, rtol=1e-8, E=None, S=None, want_E=True):
        """All-port solve: TE10 incidence on every port; returns (E, S, info)
        with S[i][j] the TE10 amplitude received on port i from port j minus
        the incident unit wave."""
        npt = self.nports
        if E is None and want_E:
            E = np.zeros((self.ne, npt), dtype=np.complex128)
        if S is None:
            S = np.zeros((npt, npt), dtype=np.complex128)
        iters = np.zeros(npt, dtype=np.int32)
        relres = np.zeros(npt, dtype=np.float64)
        info = SolveInfo(iters.ctypes.data, relres.ctypes.data)
        rc = lib().mx_solve_ports(self._h, float(rtol), _ptr(E), _ptr(S), ct.byref(info))
        _check(rc, allow=(MX_ENOTCONV,))
        return E, S, _info_dict(info, iters, relres, rc)

    def gradient(self, S_meas, w, alpha, grad=None):
        """Cost J and complex gradient dJ/dRe eps + j dJ/dIm eps (per vertex)
        for the transmitters/receivers of the last solve; returns (J, grad, info)."""
        S_meas = np.ascontiguousarray(S_meas, dtype=np.complex128)
        w = np.ascontiguousarray(w, dtype=np.float64)
        if grad is None:
            grad = np.zeros(self.sizes().nv, np.complex128)
        ntx = S_meas.shape[1]
        iters = np.zeros(ntx, dtype=np.int32)
        relres = np.zeros(ntx, dtype=np.float64)
        info = SolveInfo(iters.ctypes.data, relres.ctypes.data)
        J = ct.c_double(0.0)
        rc = lib().mx_gradient(self._h, _ptr(S_meas), _ptr(w), float(alpha), _ptr(grad), ct.byref(J), ct.byref(info))
        _check(rc, allow=(MX_ENOTCONV,))
        return J.value, grad, {"iters": iters, "relres": relres, "iters_max": info.iters_max,
                               "converged": rc == MX_OK}

    def solve_rhs(self, b, rtol=1e-8, x=None):
        nrhs = b.shape[1]
        if not _is_torch(b):
            b = np.ascontiguousarray(b, dtype=np.complex128)
        if x is None:
            x = np.zeros((self.ne, nrhs), dtype=np.complex128)
        iters = np.zeros(nrhs, dtype=np.int32)
        relres = np.zeros(nrhs, dtype=np.float64)
        info = SolveInfo(iters.ctypes.data, relres.ctypes.data)
        rc = lib().mx_solve_rhs(self._h, _ptr(b), nrhs, float(rtol), _ptr(x), ct.byref(info))
        _check(rc, allow=(MX_ENOTCONV,))
        return x, _info_dict(info, iters, relres, rc)

    def apply_operator(self, X, Y=None):
        X2 = X if _is_torch(X) else np.ascontiguousarray(X, dtype=np.complex128)
        if Y is None:
            Y = np.zeros_like(X2) if not _is_torch(X2) else X2.clone()
        _check(lib().mx_apply_operator(self._h, _ptr(X2), _ptr(Y), X2.shape[1]))
        return Y

    def apply_preconditioner(self, X, Z=None):
        X2 = X if _is_torch(X) else np.ascontiguousarray(X, dtype=np.complex128)
        if Z is None:
            Z = np.zeros_like(X2) if not _is_torch(X2) else X2.clone()
        _check(lib().mx_apply_preconditioner(self._h, _ptr(X2), _ptr(Z), X2.shape[1]))
        return Z

    def apply_preconditioner_noalloc(self, X, Z):
        """Z = M^{-1} X (one-level) for device tensors X, Z [ne][nrhs]
        complex128, with no device allocation; enqueued on the context's
        stream without synchronising."""
        if not (_is_torch(X) and _is_torch(Z)):
            raise ValueError("X and Z must be device tensors")
        _check(lib().mx_apply_preconditioner_noalloc(self._h, _ptr(X), _ptr(Z), X.shape[1]))
        return Z

    # -- inspection ------------------------------------------------------------
    def sizes(self):
        s = Sizes()
        _check(lib().mx_get_sizes(self._h, ct.byref(s)))
        return s

    def topology(self):
        s = self.sizes()
        edges = np.zeros((s.ne, 2), np.int32)
        t2e = np.zeros((s.nt, 6), np.int32)
        rp = np.zeros(s.ne + 1, np.int64)
        col = np.zeros(s.nnz, np.int32)
        _check(lib().mx_get_topology(self._h, _ptr(edges), _ptr(t2e), _ptr(rp), _ptr(col)))
        return edges, t2e, rp, col

    def matrix_values(self):
        v = np.zeros(self.sizes().nnz, np.complex128)
        _check(lib().mx_get_matrix_values(self._h, _ptr(v)))
        return v

    def partition(self):
        s = self.sizes()
        part = np.zeros(s.nt, np.int32)
        dp = np.zeros(s.nsub + 1, np.int64)
        dofs = np.zeros(s.sum_ni, np.int32)
        w = np.zeros(s.sum_ni, np.int32)
        col = np.zeros(s.nsub, np.int32)
        _check(lib().mx_get_partition(self._h, _ptr(part), _ptr(dp), _ptr(dofs), _ptr(w), _ptr(col)))
        return part, dp, dofs, w, col

    def local_matrix(self, i):
        dp = self.partition()[1]
        n = int(dp[i + 1] - dp[i])
        B = np.zeros((n, n), np.complex128)
        _check(lib().mx_get_local_matrix(self._h, int(i), _ptr(B)))
        return B

    # -- learned coarse correction -------------------------------------------
    def coarse_init(self, seed=0):
        _check(lib().mx_coarse_init(self._h, int(seed)))

    def coarse_weights(self):
        n = lib().mx_coarse_num_params()
        th = np.zeros(n, np.float32)
        sx, sy = ct.c_double(), ct.c_double()
        _check(lib().mx_coarse_get_weights(self._h, _ptr(th), n, ct.byref(sx), ct.byref(sy)))
        return th, sx.value, sy.value

    def coarse_set_weights(self, theta, in_scale=1.0, out_scale=1.0):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        _check(lib().mx_coarse_set_weights(self._h, _ptr(th), th.size, float(in_scale), float(out_scale)))

    def coarse_features(self, v):
        v2 = v if _is_torch(v) else np.ascontiguousarray(v, dtype=np.complex128)
        nrhs = v2.shape[1]
        X = np.zeros((nrhs, self.sizes().nsub, 384), np.float32)
        _check(lib().mx_coarse_features(self._h, _ptr(v2), nrhs, _ptr(X)))
        return X

    def coarse_forward(self, X):
        X = np.ascontiguousarray(X, dtype=np.float32)
        out = np.zeros_like(X)
        _check(lib().mx_coarse_forward(self._h, _ptr(X), X.shape[0], _ptr(out)))
        return out

    def coarse_hidden(self, X):
        """(H [5, G, nsub, 256], out [G, nsub, 384]): hidden activations of the
        four MLP layers and the first message-passing layer, and the outputs."""
        X = np.ascontiguousarray(X, dtype=np.float32)
        H = np.zeros((5,) + X.shape[:2] + (256,), np.float32)
        out = np.zeros_like(X)
        _check(lib().mx_coarse_hidden(self._h, _ptr(X), X.shape[0], _ptr(H), _ptr(out)))
        return H, out

    def coarse_adam_step(self, grad, lr):
        g = grad if _is_torch(grad) else np.ascontiguousarray(grad, dtype=np.float32)
        _check(lib().mx_coarse_adam_step(self._h, _ptr(g), int(np.prod(g.shape)), float(lr)))

    def coarse_loss_grad(self, X, Y):
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.ascontiguousarray(Y, dtype=np.float32)
        g = np.zeros(lib().mx_coarse_num_params(), np.float32)
        loss = ct.c_double()
        _check(lib().mx_coarse_loss_grad(self._h, _ptr(X), _ptr(Y), X.shape[0], ct.byref(loss), _ptr(g)))
        return loss.value, g

    def coarse_collect(self, pos, mom, snap_every=3, max_snapshots=20, rtol_exact=1e-12):
        tx, keep = _sources(pos, mom)
        n = ct.c_int32()
        _check(lib().mx_coarse_collect(self._h, ct.byref(tx), int(snap_every), int(max_snapshots),
                                       float(rtol_exact), ct.byref(n)))
        return n.value

    def coarse_clear(self):
        _check(lib().mx_coarse_clear(self._h))

    def coarse_train(self, epochs, batch_graphs=8, lr=1e-3, seed=0):
        hist = np.zeros(epochs, np.float64)
        _check(lib().mx_coarse_train(self._h, int(epochs), int(batch_graphs), float(lr), int(seed), _ptr(hist)))
        return hist

    def point_functionals(self, pos, mom):
        s, keep = _sources(pos, mom)
        R = np.zeros((self.ne, s.n), np.complex128)
        _check(lib().mx_point_functionals(self._h, ct.byref(s), _ptr(R)))
        return R
