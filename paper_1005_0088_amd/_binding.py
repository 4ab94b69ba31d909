"""ctypes binding of libndrho.so (argument marshalling only)."""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libndrho.so")

FP64, MIXED_FP32, MIXED_BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "mixed_fp32": MIXED_FP32, "mixed_bf16x3": MIXED_BF16X3}

STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "ENOTSPD", -4: "ESINGULAR", -5: "EDEVICE",
                -6: "ESTATE", -7: "EUNSUPPORTED"}


class NdrhoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(code, "?"), code, msg))
        self.code = code
        self.name = STATUS_NAMES.get(code, "?")


class Options(C.Structure):
    _fields_ = [("leaf_rows", C.c_int32), ("precision", C.c_int32), ("pole_batch", C.c_int32),
                ("mem_fraction", C.c_double), ("verbose", C.c_int32), ("fp64_poles", C.c_int32),
                ("fp64_pole_im", C.c_double), ("fp64_far_poles", C.c_int32), ("use_graph", C.c_int32),
                ("gemm_variant", C.c_int32), ("fp64_small_tiles", C.c_int32),
                ("split_streams", C.c_int32), ("long_tail", C.c_double), ("small_fronts", C.c_int32),
                ("pivot_variant", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("n_fronts", C.c_int32), ("n_levels", C.c_int32),
                ("max_front_j", C.c_int32), ("max_front_u", C.c_int32), ("root_j", C.c_int32),
                ("n_poles", C.c_int32), ("pole_batch", C.c_int32), ("flops_per_pole", C.c_double),
                ("flops_exec_per_pole", C.c_double), ("bytes_per_pole", C.c_double),
                ("factor_bytes_per_pole", C.c_double), ("workspace_bytes", C.c_double),
                ("last_ms", C.c_double), ("launches_per_pass", C.c_int64), ("n_fp64_poles", C.c_int32),
                ("precision", C.c_int32), ("split_passes", C.c_int32)]


_P = C.c_void_p
_I32P = C.POINTER(C.c_int32)
_I64P = C.POINTER(C.c_int64)
_DP = C.POINTER(C.c_double)

# (name, restype, argtypes) of every exported symbol declared in include/ndrho.h
SIGNATURES = [
    ("ndrho_default_options", C.c_int, [C.POINTER(Options)]),
    ("ndrho_create", C.c_int, [C.POINTER(_P), C.c_int, _P, C.POINTER(Options)]),
    ("ndrho_destroy", C.c_int, [_P]),
    ("ndrho_last_error", C.c_char_p, [_P]),
    ("ndrho_set_structure", C.c_int, [_P, C.c_int64, _I64P, _I32P, _DP, _DP, _DP, _I32P]),
    ("ndrho_set_structure_periodic", C.c_int, [_P, C.c_int64, _I64P, _I32P, _DP, _DP, _DP, _DP, _I32P]),
    ("ndrho_update_values", C.c_int, [_P, C.c_int32, _DP, _DP]),
    ("ndrho_set_poles", C.c_int, [_P, C.c_int32, C.c_double, C.c_double, C.c_int32]),
    ("ndrho_set_shifts", C.c_int, [_P, C.c_int32, C.c_int32, _DP, _DP, _DP, C.c_int32]),
    ("ndrho_density_matrix", C.c_int, [_P, C.c_int32, _P, C.c_int32]),
    ("ndrho_density_matrix_noalloc", C.c_int, [_P, C.c_int32, _P]),
    ("ndrho_energy_density_matrix", C.c_int, [_P, C.c_int32, _P, _P, C.c_int32]),
    ("ndrho_energy_density_matrix_batch", C.c_int, [_P, _I32P, C.c_int32, C.POINTER(_P), C.POINTER(_P), C.c_int32]),
    ("ndrho_eigenstates", C.c_int, [_P, C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_int32, C.c_double, _DP, _DP,
                                    _I32P, _DP]),
    ("ndrho_green_traces", C.c_int, [_P, C.c_int32, C.c_int32, _P, _P, _P, _P]),
    ("ndrho_find_mu", C.c_int, [_P, C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int32), _P]),
    ("ndrho_density_matrix_batch", C.c_int, [_P, _I32P, C.c_int32, C.POINTER(_P), C.c_int32]),
    ("ndrho_autotune", C.c_int, [_P, _I32P, C.c_int32, C.c_char_p]),
    ("ndrho_structure_stats", C.c_int, [_P, C.c_int32, C.POINTER(Stats)]),
    ("ndrho_stats", C.c_int, [_P, _DP, _DP, _DP]),
    ("ndrho_profile", C.c_int, [_P, C.c_int32]),
    ("ndrho_profile_read", C.c_int, [_P, _DP, _DP, _I64P]),
    ("ndrho_profile_read_depth", C.c_int, [_P, _DP]),
    ("ndrho_profile_read_bytes", C.c_int, [_P, _DP]),
    ("ndrho_device_alloc", C.c_int, [_P, C.c_int64, C.POINTER(_P)]),
    ("ndrho_device_free", C.c_int, [_P, _P]),
    ("ndrho_device_to_host", C.c_int, [_P, _P, _P, C.c_int64]),
    ("ndrho_device_copy", C.c_int, [_P, _P, _P, C.c_int64]),
    ("ndrho_cf_poles", C.c_int, [C.c_int32, _DP, _DP]),
    ("ndrho_plan_create", C.c_int, [C.c_int64, _I64P, _I32P, _DP, _DP, C.c_int32, C.c_double, C.POINTER(_P)]),
    ("ndrho_plan_destroy", C.c_int, [_P]),
    ("ndrho_plan_last_error", C.c_char_p, []),
    ("ndrho_plan_counts", C.c_int, [_P, _I64P]),
    ("ndrho_plan_export", C.c_int, [_P, _I32P, _I32P, _I32P, _I64P, _I32P, _I32P, _I64P, _I32P, _I32P]),
    ("ndrho_plan_slots", C.c_int, [_P, _I64P, _I64P, _I64P]),
    ("ndrho_plan_program", C.c_int, [_P, _I64P, _I32P, _I32P, _DP, _I64P]),
    ("ndrho_plan_model", C.c_int, [_P, _DP, _DP]),
]

_lib = None


def load_library():
    """Load libndrho.so (built by paper_1005_0088_amd.build); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path):
            raise ImportError("libndrho.so is not built: run `python -m paper_1005_0088_amd.build`")
        lib = C.CDLL(lib_path)
        for name, res, args in SIGNATURES:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def _csr(row_ptr, col):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    return rp, cl


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def cf_poles(n_poles):
    """Continued-fraction poles z_p and residues R_p computed by the library."""
    lib = load_library()
    z = np.empty(n_poles)
    r = np.empty(n_poles)
    rc = lib.ndrho_cf_poles(int(n_poles), _ptr(z, C.c_double), _ptr(r, C.c_double))
    if rc:
        raise NdrhoError(rc, lib.ndrho_plan_last_error().decode() or lib.ndrho_last_error(None).decode())
    return z, r


class Plan:
    """Host-only nested dissection + symbolic analysis (for inspection and tests)."""

    def __init__(self, n, row_ptr, col, coords=None, leaf_rows=32, long_tail=0.0, cell=None):
        self._lib = load_library()
        rp, cl = _csr(row_ptr, col)
        xyz = _f64(coords)
        cl3 = None if cell is None else _f64(np.asarray(cell, dtype=np.float64).reshape(3))
        h = C.c_void_p()
        rc = self._lib.ndrho_plan_create(int(n), _ptr(rp, C.c_int64), _ptr(cl, C.c_int32),
                                         _ptr(xyz, C.c_double), _ptr(cl3, C.c_double), int(leaf_rows),
                                         float(long_tail), C.byref(h))
        if rc:
            raise NdrhoError(rc, self._lib.ndrho_plan_last_error().decode())
        self._h = h
        self.n = int(n)
        cnt = np.zeros(7, dtype=np.int64)
        self._lib.ndrho_plan_counts(self._h, _ptr(cnt, C.c_int64))
        (self.n_fronts, self.n_levels, self.sum_u, self.nnz, self.panel_total, self.max_j,
         self.max_u) = (int(x) for x in cnt)

    def export(self):
        nf, su = self.n_fronts, self.sum_u
        out = {"perm": np.empty(self.n, np.int32), "parent": np.empty(nf, np.int32),
               "depth": np.empty(nf, np.int32), "j0": np.empty(nf, np.int64), "nj": np.empty(nf, np.int32),
               "nu": np.empty(nf, np.int32), "u_off": np.empty(nf, np.int64),
               "u_rows": np.empty(max(su, 1), np.int32), "rel": np.empty(max(su, 1), np.int32)}
        self._lib.ndrho_plan_export(self._h, _ptr(out["perm"], C.c_int32), _ptr(out["parent"], C.c_int32),
                                    _ptr(out["depth"], C.c_int32), _ptr(out["j0"], C.c_int64),
                                    _ptr(out["nj"], C.c_int32), _ptr(out["nu"], C.c_int32),
                                    _ptr(out["u_off"], C.c_int64), _ptr(out["u_rows"], C.c_int32),
                                    _ptr(out["rel"], C.c_int32))
        out["u_rows"] = out["u_rows"][:su]
        out["rel"] = out["rel"][:su]
        return out

    def slots(self):
        out = np.empty(self.nnz, np.int64)
        asm = np.empty(self.nnz, np.int64)
        poff = np.empty(self.n_fronts, np.int64)
        self._lib.ndrho_plan_slots(self._h, _ptr(out, C.c_int64), _ptr(asm, C.c_int64), _ptr(poff, C.c_int64))
        return out, asm, poff

    def program(self):
        cnt = C.c_int64()
        self._lib.ndrho_plan_program(self._h, C.byref(cnt), None, None, None, None)
        m = cnt.value
        kind = np.empty(m, np.int32)
        depth = np.empty(m, np.int32)
        flops = np.empty(m)
        items = np.empty(m, np.int64)
        self._lib.ndrho_plan_program(self._h, C.byref(cnt), _ptr(kind, C.c_int32), _ptr(depth, C.c_int32),
                                     _ptr(flops, C.c_double), _ptr(items, C.c_int64))
        return {"kind": kind, "depth": depth, "flops": flops, "items": items}

    def model(self):
        f = C.c_double()
        b = C.c_double()
        self._lib.ndrho_plan_model(self._h, C.byref(f), C.byref(b))
        return f.value, b.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.ndrho_plan_destroy(h)
            self._h = None


class DeviceBuffer:
    """float64 device array owned by a Context (for device-resident outputs)."""

    def __init__(self, ctx, n):
        self.ctx = ctx
        self.n = int(n)
        p = C.c_void_p()
        ctx._check(ctx._lib.ndrho_device_alloc(ctx._h, 8 * max(1, self.n), C.byref(p)))
        self.ptr = p.value

    def numpy(self):
        out = np.empty(self.n, dtype=np.float64)
        self.ctx._check(self.ctx._lib.ndrho_device_to_host(self.ctx._h, out.ctypes.data_as(C.c_void_p),
                                                           C.c_void_p(self.ptr), 8 * self.n))
        return out

    def copy_from(self, other):
        """Device-to-device copy of another buffer of the same size (plain copy kernel)."""
        if other.n != self.n:
            raise ValueError("size mismatch")
        self.ctx._check(self.ctx._lib.ndrho_device_copy(self.ctx._h, C.c_void_p(self.ptr), C.c_void_p(other.ptr),
                                                        8 * self.n))

    def free(self):
        if self.ptr and self.ctx._h:
            self.ctx._lib.ndrho_device_free(self.ctx._h, C.c_void_p(self.ptr))
        self.ptr = None


class Context:
    """One ndrho context on a HIP device.

    stream: an integer hipStream_t handle created with the same HIP runtime
    as libndrho.so, or None (the context creates its own stream).
    """

    def __init__(self, device=0, stream=None, leaf_rows=32, pole_batch=0, mem_fraction=0.8, precision="fp64",
                 fp64_poles=None, fp64_pole_im=None, use_graph=True, gemm_variant=-1, fp64_far_poles=None,
                 fp64_small_tiles=-1, split_streams=0, long_tail=0.0, verbose=0, small_fronts=0,
                 pivot_variant=0):
        self._lib = load_library()
        opt = Options()
        self._lib.ndrho_default_options(C.byref(opt))
        opt.leaf_rows = int(leaf_rows)
        opt.pole_batch = int(pole_batch)
        opt.mem_fraction = float(mem_fraction)
        opt.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        if fp64_poles is not None:
            opt.fp64_poles = int(fp64_poles)
        if fp64_pole_im is not None:
            opt.fp64_pole_im = float(fp64_pole_im)
        if fp64_far_poles is not None:
            opt.fp64_far_poles = int(fp64_far_poles)
        opt.use_graph = int(bool(use_graph))
        opt.gemm_variant = int(gemm_variant)
        opt.fp64_small_tiles = int(fp64_small_tiles)
        opt.split_streams = int(split_streams)
        opt.long_tail = float(long_tail)
        opt.small_fronts = int(small_fronts)
        opt.pivot_variant = int(pivot_variant)
        opt.verbose = int(verbose)
        handle = None
        if stream is not None:
            handle = getattr(stream, "cuda_stream", stream)
        self._stream_obj = stream
        h = C.c_void_p()
        rc = self._lib.ndrho_create(C.byref(h), int(device), C.c_void_p(handle) if handle else None, C.byref(opt))
        if rc:
            raise NdrhoError(rc, self._lib.ndrho_last_error(None).decode())
        self._h = h
        self._nnz = {}
        self._n = {}

    def _check(self, rc):
        if rc:
            raise NdrhoError(rc, self._lib.ndrho_last_error(self._h).decode())

    def set_structure(self, n, row_ptr, col, h, s, coords=None, cell=None):
        """Register H, S (CSR); cell: None (open) or the periodic cell lengths
        along x, y, z (ndrho_set_structure_periodic)."""
        rp, cl = _csr(row_ptr, col)
        hv, sv, xyz = _f64(h), _f64(s), _f64(coords)
        sid = C.c_int32()
        if cell is None:
            self._check(self._lib.ndrho_set_structure(self._h, int(n), _ptr(rp, C.c_int64), _ptr(cl, C.c_int32),
                                                      _ptr(hv, C.c_double), _ptr(sv, C.c_double),
                                                      _ptr(xyz, C.c_double), C.byref(sid)))
        else:
            cl3 = _f64(np.asarray(cell, dtype=np.float64).reshape(3))
            self._check(self._lib.ndrho_set_structure_periodic(
                self._h, int(n), _ptr(rp, C.c_int64), _ptr(cl, C.c_int32), _ptr(hv, C.c_double),
                _ptr(sv, C.c_double), _ptr(xyz, C.c_double), _ptr(cl3, C.c_double), C.byref(sid)))
        self._nnz[sid.value] = int(rp[-1])
        self._n[sid.value] = int(n)
        return sid.value

    def update_values(self, sid, h, s):
        hv, sv = _f64(h), _f64(s)
        self._check(self._lib.ndrho_update_values(self._h, int(sid), _ptr(hv, C.c_double), _ptr(sv, C.c_double)))

    def set_poles(self, sid, mu, beta, n_poles):
        self._check(self._lib.ndrho_set_poles(self._h, int(sid), float(mu), float(beta), int(n_poles)))

    def set_shifts(self, sid, alpha, weights, add_m0=True):
        a = np.ascontiguousarray(alpha, dtype=np.complex128)
        ar = np.ascontiguousarray(a.real)
        ai = np.ascontiguousarray(a.imag)
        w = _f64(weights)
        self._check(self._lib.ndrho_set_shifts(self._h, int(sid), int(a.shape[0]), _ptr(ar, C.c_double),
                                               _ptr(ai, C.c_double), _ptr(w, C.c_double), int(bool(add_m0))))

    def device_buffer(self, n):
        return DeviceBuffer(self, n)

    def density_matrix(self, sid, out=None):
        """rho on the pattern in CSR order.  out: None (returns a new numpy
        array), a float64 numpy array, or a DeviceBuffer of nnz elements
        (filled on the device, no host copy)."""
        nnz = self._nnz[int(sid)]
        if out is None:
            out = np.empty(nnz, dtype=np.float64)
        if isinstance(out, np.ndarray):
            if out.dtype != np.float64 or out.size != nnz or not out.flags.c_contiguous:
                raise ValueError("out must be a contiguous float64 array of nnz elements")
            self._check(self._lib.ndrho_density_matrix(self._h, int(sid), out.ctypes.data_as(C.c_void_p), 0))
            return out
        if not isinstance(out, DeviceBuffer) or out.ctx is not self or out.n != nnz:
            raise ValueError("out must be a numpy array or a DeviceBuffer of nnz elements from this context")
        self._check(self._lib.ndrho_density_matrix(self._h, int(sid), C.c_void_p(out.ptr), 1))
        return out

    def density_matrix_noalloc(self, sid, out):
        """rho into a DeviceBuffer of nnz elements through the entry point that
        allocates nothing (ndrho_density_matrix_noalloc)."""
        nnz = self._nnz[int(sid)]
        if not isinstance(out, DeviceBuffer) or out.ctx is not self or out.n != nnz:
            raise ValueError("out must be a DeviceBuffer of nnz elements from this context")
        self._check(self._lib.ndrho_density_matrix_noalloc(self._h, int(sid), C.c_void_p(out.ptr)))
        return out

    def eigenstates(self, sid, xi, k, eta=1e-3, max_iter=200, tol=1e-9, vectors=True):
        """The k eigenpairs nearest xi (ndrho_eigenstates).  Returns (eps,
        C (n x k, or None), iterations, residual norms)."""
        n = self._n[int(sid)]
        eps = np.empty(int(k))
        res = np.empty(int(k))
        c = np.empty((int(k), n)) if vectors else None
        it = C.c_int32()
        self._check(self._lib.ndrho_eigenstates(self._h, int(sid), float(xi), float(eta), int(k), int(max_iter),
                                                float(tol), _ptr(eps, C.c_double),
                                                _ptr(c, C.c_double) if vectors else None, C.byref(it),
                                                _ptr(res, C.c_double)))
        return eps, (c.T.copy() if vectors else None), it.value, res

    def green_traces(self, sid, alpha):
        """Tr(G(alpha_k) S) for an array of complex shifts (see ndrho_green_traces)."""
        a = np.ascontiguousarray(alpha, dtype=np.complex128).ravel()
        re, im = np.ascontiguousarray(a.real), np.ascontiguousarray(a.imag)
        tr_re, tr_im = np.empty(a.size), np.empty(a.size)
        self._check(self._lib.ndrho_green_traces(self._h, int(sid), int(a.size), re.ctypes.data_as(C.c_void_p),
                                                 im.ctypes.data_as(C.c_void_p), tr_re.ctypes.data_as(C.c_void_p),
                                                 tr_im.ctypes.data_as(C.c_void_p)))
        return tr_re + 1j * tr_im

    def find_mu(self, sid, n_ideal, beta, n_poles, mu0=0.0, tol=1e-8, max_iter=40, retarded_step=False):
        """Chemical potential with Tr(rho S) = n_ideal (see ndrho_find_mu).
        Returns (mu, delta_n, evaluations, rho in CSR order); the structure's
        poles are left at mu."""
        nnz = self._nnz[int(sid)]
        rho = np.empty(nnz, dtype=np.float64)
        mu, dn, it = C.c_double(), C.c_double(), C.c_int32()
        self._check(self._lib.ndrho_find_mu(self._h, int(sid), float(n_ideal), float(beta), int(n_poles), float(mu0),
                                            float(tol), int(max_iter), int(bool(retarded_step)), C.byref(mu),
                                            C.byref(dn), C.byref(it),
                                            rho.ctypes.data_as(C.c_void_p)))
        return mu.value, dn.value, it.value, rho

    def energy_density_matrix(self, sid, rho_out=None, e_out=None):
        """(rho, e) on the pattern in CSR order (see ndrho_energy_density_matrix).
        Outputs: None (new numpy arrays), float64 numpy arrays, or DeviceBuffers of nnz elements."""
        nnz = self._nnz[int(sid)]
        outs = [np.empty(nnz, dtype=np.float64) if o is None else o for o in (rho_out, e_out)]
        on_dev = [isinstance(o, DeviceBuffer) for o in outs]
        if on_dev[0] != on_dev[1]:
            raise ValueError("rho_out and e_out must both be numpy arrays or both DeviceBuffers")
        for o in outs:
            if on_dev[0]:
                if o.ctx is not self or o.n != nnz:
                    raise ValueError("each DeviceBuffer must hold nnz elements from this context")
            elif o.dtype != np.float64 or o.size != nnz or not o.flags.c_contiguous:
                raise ValueError("each output must be a contiguous float64 array of nnz elements")
        ptrs = [C.c_void_p(o.ptr) if on_dev[0] else o.ctypes.data_as(C.c_void_p) for o in outs]
        self._check(self._lib.ndrho_energy_density_matrix(self._h, int(sid), ptrs[0], ptrs[1], int(on_dev[0])))
        return outs[0], outs[1]

    def energy_density_matrix_batch(self, sids):
        """(rho list, e list) of several structures in one schedule (host arrays;
        see ndrho_energy_density_matrix_batch)."""
        sids = [int(s) for s in sids]
        rhos = [np.empty(self._nnz[s], dtype=np.float64) for s in sids]
        es = [np.empty(self._nnz[s], dtype=np.float64) for s in sids]
        ids = np.asarray(sids, dtype=np.int32)
        pr = (C.c_void_p * len(sids))(*[o.ctypes.data for o in rhos])
        pe = (C.c_void_p * len(sids))(*[o.ctypes.data for o in es])
        self._check(self._lib.ndrho_energy_density_matrix_batch(self._h, ids.ctypes.data_as(_I32P), len(sids), pr,
                                                                pe, 0))
        return rhos, es

    def density_matrix_batch(self, sids, outs=None):
        """rho of several structures in one schedule (see ndrho_density_matrix_batch).
        outs: None (new numpy arrays), a list of numpy arrays, or a list of DeviceBuffers."""
        sids = [int(s) for s in sids]
        if outs is None:
            outs = [np.empty(self._nnz[s], dtype=np.float64) for s in sids]
        on_dev = all(isinstance(o, DeviceBuffer) for o in outs)
        for s, o in zip(sids, outs):
            n = o.n if isinstance(o, DeviceBuffer) else o.size
            if n != self._nnz[s] or (not on_dev and (o.dtype != np.float64 or not o.flags.c_contiguous)):
                raise ValueError("each output must hold nnz float64 values of its structure")
        ids = np.asarray(sids, dtype=np.int32)
        ptrs = (C.c_void_p * len(sids))(*[o.ptr if on_dev else o.ctypes.data for o in outs])
        self._check(self._lib.ndrho_density_matrix_batch(self._h, _ptr(ids, C.c_int32), len(sids), ptrs,
                                                         int(on_dev)))
        return outs

    def autotune(self, sids, cache_path=None):
        """Pick the fastest GEMM variant per launch for one structure or a batch."""
        ids = np.asarray([int(x) for x in (sids if hasattr(sids, "__len__") else [sids])], dtype=np.int32)
        path = cache_path.encode() if cache_path else None
        self._check(self._lib.ndrho_autotune(self._h, _ptr(ids, C.c_int32), int(ids.size), path))

    def stats(self, sid):
        st = Stats()
        self._check(self._lib.ndrho_structure_stats(self._h, int(sid), C.byref(st)))
        return {k: getattr(st, k) for k, _ in Stats._fields_}

    PHASES = ("assemble", "upward", "downward", "accumulate")

    def phase_stats(self):
        """ndrho_stats: profiled milliseconds per phase, and the algorithmic
        flops and bytes of the last evaluation."""
        ms = np.zeros(4)
        fl, by = C.c_double(), C.c_double()
        self._check(self._lib.ndrho_stats(self._h, _ptr(ms, C.c_double), C.byref(fl), C.byref(by)))
        return {"ms_per_phase": dict(zip(self.PHASES, (float(x) for x in ms))), "flops": fl.value,
                "hbm_bytes": by.value}

    KINDS = ("extadd", "assemble", "pivot_inv", "gemm", "copy", "gather", "accum", "gemm_pivot", "gemm_f32", "gemm_bf16x3",
             "small_fronts")

    def profile(self, enable=True):
        self._check(self._lib.ndrho_profile(self._h, int(bool(enable))))

    def profile_read(self):
        k = len(self.KINDS)
        ms = np.zeros(k)
        fl = np.zeros(k)
        nl = np.zeros(k, dtype=np.int64)
        self._check(self._lib.ndrho_profile_read(self._h, _ptr(ms, C.c_double), _ptr(fl, C.c_double),
                                                 _ptr(nl, C.c_int64)))
        by = np.zeros(k)
        self._check(self._lib.ndrho_profile_read_bytes(self._h, _ptr(by, C.c_double)))
        return {name: {"ms": float(ms[i]), "flops": float(fl[i]), "launches": int(nl[i]), "bytes": float(by[i])}
                for i, name in enumerate(self.KINDS)}

    def profile_read_depth(self):
        """Profiled milliseconds per kernel kind and tree depth: {kind: array over depths}
        (the last column holds launches outside the tree)."""
        nd_ = 32
        ms = np.zeros(len(self.KINDS) * nd_)
        self._check(self._lib.ndrho_profile_read_depth(self._h, _ptr(ms, C.c_double)))
        ms = ms.reshape(len(self.KINDS), nd_)
        return {name: ms[i].copy() for i, name in enumerate(self.KINDS)}

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.ndrho_destroy(h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
