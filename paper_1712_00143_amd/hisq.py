"""ctypes binding of libhisq.so (the C ABI declared in include/hisq.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Functions keep the C names; ``Lattice`` and ``PTC`` wrap the
handles.  Arrays may be numpy (host, complex128) or torch tensors on the GPU
(passed by device pointer with HISQ_DEVICE_PTR).  The library must have been
built (``paper_1712_00143_amd.build.build()``); importing this module without
it raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhisq.so")

HISQ_OK = 0
HISQ_LOSS_ENERGY = 0
HISQ_LOSS_EUCLIDEAN = 1
HISQ_ERR_ARG = -1
HISQ_ERR_HIP = -2
HISQ_ERR_OOM = -3
HISQ_ERR_STATE = -4
HISQ_ERR_RECON = -5
HISQ_ERR_NOT_CONVERGED = -6
HISQ_ERR_BREAKDOWN = -7
HISQ_ERR_IO = -8

HISQ_F64, HISQ_F32, HISQ_F16 = 0, 1, 2
HISQ_RECON_18, HISQ_RECON_12 = 18, 12
HISQ_EVEN, HISQ_ODD = 0, 1
HISQ_DEVICE_PTR, HISQ_X_IS_GUESS, HISQ_USE_GRAPH, HISQ_NO_TUNE = 1, 2, 4, 8
HISQ_STOP_STAGNATION = 16
HISQ_STREAM_LINKS = 32
HISQ_LOAD_RESULT = 64

EXPORTS = [
    "hisq_default_params", "hisq_status_string", "hisq_last_error", "hisq_create", "hisq_destroy",
    "hisq_load_links", "hisq_prepare_links", "hisq_dslash", "hisq_cg", "hisq_multishift_cg",
    "hisq_batch_cg", "hisq_ptc_create", "hisq_ptc_destroy", "hisq_ptc_set_weights",
    "hisq_ptc_get_weights", "hisq_ptc_layer_forward", "hisq_ptc_layer_backward", "hisq_ptc_apply",
    "hisq_ptc_harvest", "hisq_ptc_train", "hisq_cg_learned", "hisq_ptc_pair_count", "hisq_ptc_get_pair",
    "hisq_stream_bandwidth", "hisq_ptc_init_polynomial", "hisq_ptc_set_loss", "hisq_ptc_save", "hisq_ptc_load",
    "hisq_residual_history", "hisq_ptc_set_transport", "hisq_ptc_get_transport", "hisq_cg_noalloc",
    "hisq_dslash_shape", "hisq_ptc_set_activations", "hisq_smear_links", "hisq_fat7", "hisq_unitarize",
    "hisq_gauge_force", "hisq_gauge_action", "hisq_fermion_force_links", "hisq_fermion_force",
]


class hisq_solver_params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int), ("sloppy", ctypes.c_int),
                ("recon", ctypes.c_int), ("delta", ctypes.c_double), ("check_every", ctypes.c_int),
                ("flags", ctypes.c_int)]


class hisq_solver_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int),
                ("converged", ctypes.c_int), ("status", ctypes.c_int),
                ("true_residual", ctypes.c_double), ("time_s", ctypes.c_double),
                ("dslash_bytes", ctypes.c_double), ("flops", ctypes.c_double),
                ("t_done_s", ctypes.c_double), ("fell_back", ctypes.c_int),
                ("fcg_iters", ctypes.c_int), ("restarts", ctypes.c_int),
                ("refine_iters", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class HisqError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch carries its own HIP runtime (same soname as the system one).
        # Load it first so that the library binds to that runtime and one
        # process never runs two HIP runtimes side by side.
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -m paper_1712_00143_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        L.hisq_status_string.restype = ctypes.c_char_p
        L.hisq_default_params.restype = None
        _lib = L
    return _lib


def hisq_status_string(status: int) -> str:
    return lib().hisq_status_string(ctypes.c_int(status)).decode()


def hisq_last_error(handle=None) -> str:
    buf = ctypes.create_string_buffer(512)
    lib().hisq_last_error(handle, buf, ctypes.c_size_t(512))
    return buf.value.decode()


def _check(st, handle=None, what=""):
    if st != HISQ_OK:
        raise HisqError(st, f"{what}: {hisq_status_string(st)}: {hisq_last_error(handle)}")


def hisq_default_params(**kw) -> hisq_solver_params:
    p = hisq_solver_params()
    lib().hisq_default_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _ptr(a):
    """(pointer, is_device, keepalive) for numpy arrays or torch tensors."""
    if a is None:
        return None, False, None
    try:
        import torch
        if isinstance(a, torch.Tensor):
            if not a.is_contiguous():
                raise ValueError("tensor must be contiguous")
            return ctypes.c_void_p(a.data_ptr()), a.is_cuda, a
    except ImportError:
        pass
    arr = np.ascontiguousarray(a)
    if arr.dtype == np.complex128 or arr.dtype == np.float64:
        return arr.ctypes.data_as(ctypes.c_void_p), False, arr
    raise TypeError(f"unsupported array type {type(a)} / {getattr(a, 'dtype', None)}")


def hisq_create(dims, device=0, stream=None):
    h = ctypes.c_void_p()
    d = (ctypes.c_int * 4)(*[int(x) for x in dims])
    st = lib().hisq_create(d, ctypes.c_int(device), stream, ctypes.byref(h))
    _check(st, None, "hisq_create")
    return h


def hisq_destroy(h):
    return lib().hisq_destroy(h)


def current_stream_ptr():
    """torch's current HIP stream as a void* (None on the null stream)."""
    import torch
    s = torch.cuda.current_stream().cuda_stream
    return ctypes.c_void_p(s) if s else None


class Lattice:
    """One periodic local lattice on one GPU (a library handle)."""

    def __init__(self, dims, device=0, stream=None, use_torch_stream=False):
        self.dims = tuple(int(x) for x in dims)
        self.V = int(np.prod(self.dims))
        self.h = self.V // 2
        if use_torch_stream:
            stream = current_stream_ptr()
        self.handle = hisq_create(self.dims, device, stream)

    def close(self):
        if self.handle is not None:
            hisq_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self):
        return hisq_last_error(self.handle)

    def load_links(self, fat, lng):
        fp, fdev, k1 = _ptr(fat)
        lp, ldev, k2 = _ptr(lng)
        flags = HISQ_DEVICE_PTR if fdev else 0
        if fdev != ldev:
            raise ValueError("fat and long links must both be host or both device arrays")
        _check(lib().hisq_load_links(self.handle, fp, lp, ctypes.c_int(flags)), self.handle,
               "hisq_load_links")

    def prepare_links(self, prec, recon):
        st = lib().hisq_prepare_links(self.handle, ctypes.c_int(prec), ctypes.c_int(recon))
        _check(st, self.handle, "hisq_prepare_links")

    def dslash(self, out_parity, prec, recon, inp, out, nrhs=1, flags=0):
        ip, idev, k1 = _ptr(inp)
        op, odev, k2 = _ptr(out)
        if idev:
            flags |= HISQ_DEVICE_PTR
        st = lib().hisq_dslash(self.handle, ctypes.c_int(out_parity), ctypes.c_int(prec),
                               ctypes.c_int(recon), ip, op, ctypes.c_int(nrhs), ctypes.c_int(flags))
        _check(st, self.handle, "hisq_dslash")
        return out

    def dslash_shape(self, prec, recon, flags=0):
        """(waves, remap, cache_blocks) of the launch hisq_dslash makes."""
        w, r, c = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        _check(lib().hisq_dslash_shape(self.handle, ctypes.c_int(prec), ctypes.c_int(recon), ctypes.c_int(flags),
                                       ctypes.byref(w), ctypes.byref(r), ctypes.byref(c)),
               self.handle, "hisq_dslash_shape")
        return w.value, r.value, c.value

    def _link_out(self, like, dev):
        if dev:
            import torch
            return torch.empty_like(like)
        return np.empty((self.V, 4, 3, 3), dtype=np.complex128)

    def smear_links(self, thin, load=False, outputs=True):
        """hisq_smear_links: (fat, lng) HISQ links from thin links (numpy
        [V][4][3][3] complex128, or a device tensor of the same bytes).  load:
        the result also becomes this lattice's links; outputs=False (with
        load) returns nothing."""
        tp, tdev, k0 = _ptr(thin)
        flags = (HISQ_DEVICE_PTR if tdev else 0) | (HISQ_LOAD_RESULT if load else 0)
        if not outputs and not load:
            raise ValueError("outputs=False needs load=True")
        fat = self._link_out(thin, tdev) if outputs else None
        lng = self._link_out(thin, tdev) if outputs else None
        fp, _, k1 = _ptr(fat)
        lp, _, k2 = _ptr(lng)
        _check(lib().hisq_smear_links(self.handle, tp, fp, lp, ctypes.c_int(flags)), self.handle,
               "hisq_smear_links")
        return (fat, lng) if outputs else None

    def fat7(self, coefs, links):
        """hisq_fat7: one smearing level with (c1, c3, c5, c7, cLepage)."""
        ip, idev, k0 = _ptr(links)
        out = self._link_out(links, idev)
        op, _, k1 = _ptr(out)
        c = (ctypes.c_double * 5)(*[float(x) for x in coefs])
        _check(lib().hisq_fat7(self.handle, c, ip, op, ctypes.c_int(HISQ_DEVICE_PTR if idev else 0)),
               self.handle, "hisq_fat7")
        return out

    def unitarize(self, links):
        """hisq_unitarize: U(3) polar factor of each of the 4 V links."""
        ip, idev, k0 = _ptr(links)
        out = self._link_out(links, idev)
        op, _, k1 = _ptr(out)
        _check(lib().hisq_unitarize(self.handle, ip, op, ctypes.c_int(HISQ_DEVICE_PTR if idev else 0)),
               self.handle, "hisq_unitarize")
        return out

    def gauge_force(self, links, beta, coefs):
        """hisq_gauge_force: Symanzik force [V][4][3][3] of thin links (coefs:
        plaquette, rectangle, parallelogram weights)."""
        ip, idev, k0 = _ptr(links)
        out = self._link_out(links, idev)
        op, _, k1 = _ptr(out)
        c = (ctypes.c_double * 3)(*[float(x) for x in coefs])
        _check(lib().hisq_gauge_force(self.handle, ip, ctypes.c_double(beta), c, op,
                                      ctypes.c_int(HISQ_DEVICE_PTR if idev else 0)), self.handle, "hisq_gauge_force")
        return out

    def gauge_action(self, links, beta, coefs):
        """hisq_gauge_action: the Symanzik action of thin links."""
        ip, idev, k0 = _ptr(links)
        c = (ctypes.c_double * 3)(*[float(x) for x in coefs])
        s = ctypes.c_double(0.0)
        _check(lib().hisq_gauge_action(self.handle, ip, ctypes.c_double(beta), c, ctypes.byref(s),
                                       ctypes.c_int(HISQ_DEVICE_PTR if idev else 0)), self.handle, "hisq_gauge_action")
        return s.value

    def _ff_vectors(self, xs, n):
        try:
            import torch
            if isinstance(xs, torch.Tensor):
                if xs.numel() != n * self.h * 6 or xs.dtype != torch.float64:
                    raise ValueError("vectors: n * V/2 * 3 complex FP64 values expected")
                return xs
        except ImportError:
            pass
        return np.ascontiguousarray(np.asarray(xs, dtype=np.complex128).reshape(n, self.h, 3))

    def fermion_force_links(self, alphas, xs):
        """hisq_fermion_force_links: (OF, OL) gradients of sum alpha_k X_k^+ A X_k
        with respect to the loaded fat and long links; xs: [n][V/2][3] complex
        (numpy, or a device tensor of the same bytes)."""
        n = len(alphas)
        xa = self._ff_vectors(xs, n)
        al = (ctypes.c_double * n)(*[float(a) for a in alphas])
        xp, xdev, k0 = _ptr(xa)
        if xdev:
            import torch
            OF = torch.empty((self.V, 4, 3, 6), dtype=torch.float64, device=xa.device)
            OL = torch.empty_like(OF)
        else:
            OF, OL = self._link_out(None, False), self._link_out(None, False)
        fp, _, k1 = _ptr(OF)
        lp, _, k2 = _ptr(OL)
        _check(lib().hisq_fermion_force_links(self.handle, ctypes.c_int(n), al, xp, fp, lp,
                                              ctypes.c_int(HISQ_DEVICE_PTR if xdev else 0)),
               self.handle, "hisq_fermion_force_links")
        return OF, OL

    def fermion_force(self, links, alphas, xs):
        """hisq_fermion_force: force [V][4][3][3] on the thin links (which are
        smeared and loaded as this lattice's links first)."""
        n = len(alphas)
        ip, idev, k0 = _ptr(links)
        xa = self._ff_vectors(xs, n)
        al = (ctypes.c_double * n)(*[float(a) for a in alphas])
        xp, xdev, k1 = _ptr(xa)
        if idev != xdev:
            raise ValueError("links and vectors must both be host or both device arrays")
        out = self._link_out(links, idev)
        op, _, k2 = _ptr(out)
        _check(lib().hisq_fermion_force(self.handle, ip, ctypes.c_int(n), al, xp, op,
                                        ctypes.c_int(HISQ_DEVICE_PTR if idev else 0)),
               self.handle, "hisq_fermion_force")
        return out

    def cg(self, mass, b, x=None, params=None, raise_on_fail=True):
        """Solve (4m^2 - D_eo D_oe) x = b; returns (x, info dict)."""
        params = params or hisq_default_params()
        if x is None:
            x = np.zeros((self.h, 3), dtype=np.complex128)
        bp, bdev, k1 = _ptr(b)
        xp, xdev, k2 = _ptr(x)
        if bdev:
            params.flags |= HISQ_DEVICE_PTR
        info = hisq_solver_info()
        st = lib().hisq_cg(self.handle, ctypes.c_double(mass), bp, xp, ctypes.byref(params),
                           ctypes.byref(info))
        if raise_on_fail:
            _check(st, self.handle, "hisq_cg")
        return x, info.as_dict()

    def cg_noalloc(self, mass, b, x, params=None, raise_on_fail=True):
        """hisq_cg_noalloc: b and x device FP64 tensors of V/2 * 6 reals; the
        solver allocates no device memory.  Returns (x, info dict)."""
        params = params or hisq_default_params()
        bp, bdev, k1 = _ptr(b)
        xp, xdev, k2 = _ptr(x)
        if bdev:
            params.flags |= HISQ_DEVICE_PTR
        info = hisq_solver_info()
        st = lib().hisq_cg_noalloc(self.handle, ctypes.c_double(mass), bp, xp, ctypes.byref(params),
                                   ctypes.byref(info))
        if raise_on_fail:
            _check(st, self.handle, "hisq_cg_noalloc")
        return x, info.as_dict()

    def residual_history(self, problem=0):
        """FP64 true relative residuals at each reliable update of the last
        solve led by this handle (see hisq_residual_history)."""
        n = ctypes.c_int(0)
        _check(lib().hisq_residual_history(self.handle, ctypes.c_int(problem), None, ctypes.c_int(0),
                                           ctypes.byref(n)), self.handle, "hisq_residual_history")
        out = np.zeros(max(n.value, 1), dtype=np.float64)
        _check(lib().hisq_residual_history(self.handle, ctypes.c_int(problem),
                                           out.ctypes.data_as(ctypes.c_void_p), ctypes.c_int(n.value),
                                           ctypes.byref(n)), self.handle, "hisq_residual_history")
        return out[:n.value]

    def multishift_cg(self, mass, shifts, b, x=None, params=None, raise_on_fail=True):
        """b: [nrhs][h][3] complex (host array), or a device FP64 tensor of
        nrhs*h*6 reals with x a device tensor of nrhs*nshift*h*6 reals;
        returns (x, info list), x as [nrhs][nshift][h][3] on the host path."""
        params = params or hisq_default_params(tol=1e-8)
        shifts = np.ascontiguousarray(shifts, dtype=np.float64)
        ns = len(shifts)
        bp, bdev, k1 = _ptr(b)
        if bdev:
            if x is None:
                raise ValueError("device right-hand sides need a device x")
            nrhs = b.numel() // (self.h * 6)
            if b.numel() != nrhs * self.h * 6 or x.numel() != nrhs * ns * self.h * 6:
                raise ValueError("b must hold nrhs*h*6 and x nrhs*nshift*h*6 reals")
            xp, xdev, k2 = _ptr(x)
            if not xdev:
                raise ValueError("x must be on the device with a device b")
            params.flags |= HISQ_DEVICE_PTR
        else:
            b = np.ascontiguousarray(b, dtype=np.complex128)
            if b.ndim == 2:
                b = b[None]
            nrhs = b.shape[0]
            bp = b.ctypes.data_as(ctypes.c_void_p)
            x = np.zeros((nrhs, ns) + b.shape[1:], dtype=np.complex128)
            xp = x.ctypes.data_as(ctypes.c_void_p)
        infos = (hisq_solver_info * (nrhs * ns))()
        st = lib().hisq_multishift_cg(self.handle, ctypes.c_double(mass), ctypes.c_int(ns),
                                      shifts.ctypes.data_as(ctypes.c_void_p), ctypes.c_int(nrhs),
                                      bp, xp, ctypes.byref(params), infos)
        if raise_on_fail:
            _check(st, self.handle, "hisq_multishift_cg")
        return x, [i.as_dict() for i in infos]


class PTC:
    """Learned parallel-transport preconditioner bound to one lattice."""

    def __init__(self, lattice, chans=(1, 4, 4, 1)):
        self.lat = lattice
        self.chans = tuple(int(c) for c in chans)
        self.nlayer = len(self.chans) - 1
        self.nw = sum(9 * a * b for a, b in zip(self.chans[:-1], self.chans[1:]))
        h = ctypes.c_void_p()
        c = (ctypes.c_int * len(self.chans))(*self.chans)
        _check(lib().hisq_ptc_create(lattice.handle, ctypes.c_int(self.nlayer), c, ctypes.byref(h)),
               lattice.handle, "hisq_ptc_create")
        self.handle = h

    def close(self):
        if self.handle is not None:
            lib().hisq_ptc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, st, what):
        _check(st, self.lat.handle, what)

    def set_weights(self, weights):
        """weights: list of complex [Cout][Cin][9] arrays, layer by layer."""
        flat = np.concatenate([np.ascontiguousarray(w, dtype=np.complex128).ravel() for w in weights])
        assert flat.size == self.nw
        self._err(lib().hisq_ptc_set_weights(self.handle, flat.ctypes.data_as(ctypes.c_void_p)),
                  "hisq_ptc_set_weights")

    def init_polynomial(self, a=4.0, c=1.2, iters=30):
        """K = a (1 + c D_f^2 / lambda): the polynomial starting point; returns
        the estimated top eigenvalue lambda of -D_f^2 on even sites."""
        lam = ctypes.c_double(0.0)
        self._err(lib().hisq_ptc_init_polynomial(self.handle, ctypes.c_double(a), ctypes.c_double(c),
                                                  ctypes.c_int(iters),
                                                  ctypes.byref(lam)), "hisq_ptc_init_polynomial")
        return lam.value

    def save(self, path):
        """Checkpoint: shape, FP32 weights and Adam state (not the pairs)."""
        self._err(lib().hisq_ptc_save(self.handle, os.fsencode(path)), "hisq_ptc_save")

    def load(self, path):
        """Restore a checkpoint written by save() from a network of this shape."""
        self._err(lib().hisq_ptc_load(self.handle, os.fsencode(path)), "hisq_ptc_load")

    def set_loss(self, loss):
        """HISQ_LOSS_ENERGY (the default) or HISQ_LOSS_EUCLIDEAN."""
        self._err(lib().hisq_ptc_set_loss(self.handle, ctypes.c_int(loss)), "hisq_ptc_set_loss")

    def set_transport(self, prec, recon):
        """Link format of the transports: (HISQ_F32, 18) or (HISQ_F16, 12);
        used by every later call of the network, training and inference."""
        self._err(lib().hisq_ptc_set_transport(self.handle, ctypes.c_int(prec), ctypes.c_int(recon)),
                  "hisq_ptc_set_transport")

    def set_activations(self, prec):
        """Inference activation storage: HISQ_F32 (default) or HISQ_F16."""
        self._err(lib().hisq_ptc_set_activations(self.handle, ctypes.c_int(prec)), "hisq_ptc_set_activations")

    def get_transport(self):
        p, r = ctypes.c_int(0), ctypes.c_int(0)
        self._err(lib().hisq_ptc_get_transport(self.handle, ctypes.byref(p), ctypes.byref(r)),
                  "hisq_ptc_get_transport")
        return p.value, r.value

    def get_weights(self):
        flat = np.zeros(self.nw, dtype=np.complex128)
        self._err(lib().hisq_ptc_get_weights(self.handle, flat.ctypes.data_as(ctypes.c_void_p)),
                  "hisq_ptc_get_weights")
        out, o = [], 0
        for a, b in zip(self.chans[:-1], self.chans[1:]):
            out.append(flat[o:o + 9 * a * b].reshape(b, a, 9))
            o += 9 * a * b
        return out

    def layer_forward(self, layer, inp, out):
        ip, _, k1 = _ptr(inp)
        op, _, k2 = _ptr(out)
        self._err(lib().hisq_ptc_layer_forward(self.handle, ctypes.c_int(layer), ip, op,
                                               ctypes.c_int(HISQ_DEVICE_PTR)), "hisq_ptc_layer_forward")

    def layer_backward(self, layer, inp, gout, gin=None):
        """Returns the weight gradient [Cout][Cin][9] (complex, host)."""
        ip, _, k1 = _ptr(inp)
        gp, _, k2 = _ptr(gout)
        gi, _, k3 = _ptr(gin)
        a, b = self.chans[layer], self.chans[layer + 1]
        gw = np.zeros((b, a, 9), dtype=np.complex128)
        self._err(lib().hisq_ptc_layer_backward(self.handle, ctypes.c_int(layer), ip, gp, gi,
                                                gw.ctypes.data_as(ctypes.c_void_p),
                                                ctypes.c_int(HISQ_DEVICE_PTR)), "hisq_ptc_layer_backward")
        return gw

    def apply(self, r, z):
        rp, _, k1 = _ptr(r)
        zp, _, k2 = _ptr(z)
        self._err(lib().hisq_ptc_apply(self.handle, rp, zp, ctypes.c_int(HISQ_DEVICE_PTR)), "hisq_ptc_apply")

    def harvest(self, lattice, mass, b, every=10, maxpairs=64):
        b = np.ascontiguousarray(b, dtype=np.complex128)
        n = ctypes.c_int(0)
        self._err(lib().hisq_ptc_harvest(self.handle, lattice.handle, ctypes.c_double(mass),
                                         b.ctypes.data_as(ctypes.c_void_p), ctypes.c_int(every),
                                         ctypes.c_int(maxpairs), ctypes.byref(n)), "hisq_ptc_harvest")
        return n.value

    def pair_count(self):
        n = ctypes.c_int(0)
        self._err(lib().hisq_ptc_pair_count(self.handle, ctypes.byref(n)), "hisq_ptc_pair_count")
        return n.value

    def get_pair(self, index, h):
        r = np.zeros((h, 3), dtype=np.complex128)
        e = np.zeros((h, 3), dtype=np.complex128)
        self._err(lib().hisq_ptc_get_pair(self.handle, ctypes.c_int(index), r.ctypes.data_as(ctypes.c_void_p),
                                          e.ctypes.data_as(ctypes.c_void_p)), "hisq_ptc_get_pair")
        return r, e

    def train(self, steps, batch=8, lr=1e-3, seed=0):
        losses = np.zeros(max(steps, 1))
        self._err(lib().hisq_ptc_train(self.handle, ctypes.c_int(steps), ctypes.c_int(batch),
                                       ctypes.c_double(lr), ctypes.c_ulonglong(seed),
                                       losses.ctypes.data_as(ctypes.c_void_p)), "hisq_ptc_train")
        return losses[:steps]

    def cg_learned(self, lattice, mass, b, x=None, params=None, raise_on_fail=True):
        params = params or hisq_default_params()
        if x is None:
            x = np.zeros((lattice.h, 3), dtype=np.complex128)
        bp, bdev, k1 = _ptr(b)
        xp, _, k2 = _ptr(x)
        if bdev:
            params.flags |= HISQ_DEVICE_PTR
        info = hisq_solver_info()
        st = lib().hisq_cg_learned(lattice.handle, self.handle, ctypes.c_double(mass), bp, xp,
                                   ctypes.byref(params), ctypes.byref(info))
        if raise_on_fail:
            _check(st, lattice.handle, "hisq_cg_learned")
        return x, info.as_dict()


def stream_bandwidth(device=0, stream=None, nbytes=1 << 30, reps=10):
    """Practical HBM ceilings (read-only, copy) in GB/s from the library's
    streaming kernels."""
    r, c = ctypes.c_double(), ctypes.c_double()
    st = lib().hisq_stream_bandwidth(ctypes.c_int(device), stream, ctypes.c_size_t(nbytes), ctypes.c_int(reps),
                                     ctypes.byref(r), ctypes.byref(c))
    _check(st, None, "hisq_stream_bandwidth")
    return r.value, c.value


def hisq_batch_cg(lattices, masses, bs, params=None, raise_on_fail=True):
    """Batched CG over several Lattice objects; returns (xs, infos)."""
    n = len(lattices)
    params = params or hisq_default_params()
    hs = (ctypes.c_void_p * n)(*[l.handle.value for l in lattices])
    ms = np.ascontiguousarray(masses, dtype=np.float64)
    bs = [np.ascontiguousarray(b, dtype=np.complex128) for b in bs]
    xs = [np.zeros_like(b) for b in bs]
    bp = (ctypes.c_void_p * n)(*[b.ctypes.data for b in bs])
    xp = (ctypes.c_void_p * n)(*[x.ctypes.data for x in xs])
    infos = (hisq_solver_info * n)()
    st = lib().hisq_batch_cg(ctypes.c_int(n), hs, ms.ctypes.data_as(ctypes.c_void_p), bp, xp,
                             ctypes.byref(params), infos)
    if raise_on_fail:
        _check(st, lattices[0].handle, "hisq_batch_cg")
    return xs, [i.as_dict() for i in infos]
