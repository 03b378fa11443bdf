"""Python binding of libems.so, the MI355X multiple-scattering operator library.

Argument marshalling only: every step of the operator runs in the HIP
kernels of ``csrc/``.  Torch supplies device memory and the stream.  Importing
this module fails loudly when the compiled library is missing.

Names follow include/ems.h.  Coefficient vectors are complex128 torch tensors
of shape [nrhs, n_coeff] on the current CUDA (HIP) device, per particle laid
out as [alpha_{-p..p}, beta_{-p..p}].
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# torch ships a HIP runtime of its own next to the one the library links.
# torch's is loaded first, as in every GPU run of the library: with the
# library's runtime loaded ahead of it, the library's runtime saw no device.
try:
    import torch  # noqa: F401
except ImportError:  # host-only use (node tables, reflection, S-matrices)
    pass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libems.so")

EMS_PART_FREE = 1
EMS_PART_REFL = 2
EMS_PART_S = 4
EMS_PART_IDENTITY = 8
EMS_APPLY_ALL = 15
EMS_MIXED = 256
# plane-wave kinds: P / SV sent from the particle side (host), P / SV sent
# from the substrate (transmitted into the host)
WAVE_P, WAVE_SV, WAVE_P_SUBSTRATE, WAVE_SV_SUBSTRATE = 0, 1, 2, 3
EMS_OK = 0
EMS_NOT_CONVERGED = 1


class EmsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ems error {code}: {msg}")
        self.code = code


class NotConvergedError(RuntimeError):
    """A solve inside a composite call (misfit and gradient) stopped at its
    iteration limit before reaching the tolerance; ``info`` is its report."""

    def __init__(self, which, info):
        super().__init__(f"{which} solve did not converge: {info['iters']} iterations, "
                         f"relative residual {info['relres']:.3e}")
        self.which = which
        self.info = info


class Medium(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_double), ("mu", ctypes.c_double), ("rho", ctypes.c_double)]


class Media(ctypes.Structure):
    _fields_ = [("host", Medium), ("substrate", Medium), ("omega", ctypes.c_double)]


class Sommerfeld(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q", ctypes.c_int32), ("t_max", ctypes.c_double),
                ("delta", ctypes.c_double), ("panel_scale", ctypes.c_double),
                ("nodes", ctypes.POINTER(ctypes.c_double)), ("panel_order", ctypes.c_int32),
                ("tail_factor", ctypes.c_double), ("depth_cut", ctypes.c_double)]


class PointSource(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("alpha1", ctypes.c_double),
                ("alpha2", ctypes.c_double)]


class PlaneWave(ctypes.Structure):
    _fields_ = [("wave", ctypes.c_int32), ("angle", ctypes.c_double)]


class SolverOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int32), ("maxit", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("inner_tol", ctypes.c_double),
                ("precond", ctypes.c_int32), ("block", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("relres", ctypes.c_double),
                ("seconds", ctypes.c_double), ("restart", ctypes.c_int32),
                ("precond_seconds", ctypes.c_double), ("reorth", ctypes.c_int32)]


class Fmm(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("leaf", ctypes.c_int32), ("top_boxes", ctypes.c_int32),
                ("digits", ctypes.c_double)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int32),
                ("total_ms", ctypes.c_double), ("flops", ctypes.c_double)]


class BuildInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("p_max", ctypes.c_int32), ("n_coeff", ctypes.c_int64),
                ("q", ctypes.c_int32), ("t_max", ctypes.c_double), ("n_pairs", ctypes.c_int64),
                ("fmm_levels", ctypes.c_int32), ("fmm_m2l", ctypes.c_int64),
                ("kp", ctypes.c_double), ("ks", ctypes.c_double), ("kpb", ctypes.c_double),
                ("ksb", ctypes.c_double), ("somm_kept", ctypes.c_double),
                ("mixed_near_fp64", ctypes.c_int32), ("mixed_somm_fp64", ctypes.c_int32)]


PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "ems_create": ([ctypes.POINTER(P)], I32),
        "ems_destroy": ([P], None),
        "ems_last_error": ([P], ctypes.c_char_p),
        "ems_set_media": ([P, ctypes.POINTER(Media)], I32),
        "ems_set_particles": ([P, I32, P, P, P], I32),
        "ems_set_smatrices": ([P, P, P], I32),
        "ems_smatrix_disk": ([ctypes.POINTER(Media), D, I32, I32, P], I32),
        "ems_smatrix_shapes": ([P, P, P, P, P, I32, D, P, P], I32),
        "ems_set_smatrices_rotated": ([P, I32, P, P, P, P], I32),
        "ems_set_sommerfeld": ([P, ctypes.POINTER(Sommerfeld)], I32),
        "ems_build": ([P, P], I32),
        "ems_get_info": ([P, ctypes.POINTER(BuildInfo)], I32),
        "ems_apply": ([P, P, P, I32, I32, P], I32),
        "ems_apply_adjoint": ([P, P, P, I32, I32, P], I32),
        "ems_incident": ([P, ctypes.POINTER(PlaneWave), I32, P, P], I32),
        "ems_solve": ([P, P, P, I32, ctypes.POINTER(SolverOpts), ctypes.POINTER(SolveInfo), P], I32),
        "ems_solve_adjoint": ([P, P, P, I32, ctypes.POINTER(SolverOpts), ctypes.POINTER(SolveInfo),
                               P], I32),
        "ems_eval_scattered": ([P, P, I32, I32, P, P, P], I32),
        "ems_eval_background": ([P, ctypes.POINTER(PlaneWave), I32, I32, P, P, P], I32),
        "ems_incident_point": ([P, ctypes.POINTER(PointSource), I32, P, P], I32),
        "ems_eval_background_point": ([P, ctypes.POINTER(PointSource), I32, I32, P, P, P], I32),
        "ems_eval_scattered_adjoint": ([P, P, I32, I32, P, P, P], I32),
        "ems_autotune": ([P, I32, ctypes.POINTER(ctypes.c_int32), P], I32),
        "ems_apply_graph": ([P, P, P, I32, I32, I32, P], I32),
        "ems_param_vjp": ([P, ctypes.POINTER(PlaneWave), I32, P, P, I32, P, P, P,
                           ctypes.POINTER(ctypes.c_double), P], I32),
        "ems_sommerfeld_nodes": ([ctypes.POINTER(Media), ctypes.POINTER(Sommerfeld), I32, P, P,
                                  ctypes.POINTER(I32), P, ctypes.POINTER(D)], I32),
        "ems_sommerfeld_depth_cuts": ([ctypes.POINTER(Media), ctypes.POINTER(Sommerfeld), I32, P,
                                       P, I32, P, P, P, ctypes.POINTER(D)], I32),
        "ems_reflection": ([ctypes.POINTER(Media), D, D, P], I32),
        "ems_profile": ([P, I32], I32),
        "ems_set_fmm": ([P, ctypes.POINTER(Fmm)], I32),
        "ems_profile_read": ([P, ctypes.POINTER(KernelTime), I32, ctypes.POINTER(I32)], I32),
        "ems_set_precond": ([P, I32], I32),
        "ems_precond_apply": ([P, P, P, I32, I32, ctypes.POINTER(I32), ctypes.POINTER(I32),
                               ctypes.POINTER(D), P], I32),
        "ems_solve_history": ([P, ctypes.POINTER(D), I32, ctypes.POINTER(I32)], I32),
        "ems_set_progress": ([P, PROGRESS_FN, I32, P], I32),
        "ems_apply_noalloc": ([P, P, P, I32, I32, P], I32),
        "ems_set_exponentials": ([P, I32], I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()
EXPORTED = ("ems_create", "ems_destroy", "ems_last_error", "ems_set_media", "ems_set_particles",
            "ems_set_smatrices", "ems_smatrix_disk", "ems_smatrix_shapes", "ems_set_smatrices_rotated",
            "ems_set_sommerfeld",
            "ems_build",
            "ems_get_info", "ems_apply", "ems_apply_adjoint", "ems_incident", "ems_solve",
            "ems_solve_adjoint", "ems_eval_scattered_adjoint", "ems_param_vjp", "ems_autotune",
            "ems_apply_graph",
            "ems_eval_scattered", "ems_eval_background", "ems_incident_point",
            "ems_eval_background_point", "ems_sommerfeld_nodes",
            "ems_sommerfeld_depth_cuts",
            "ems_reflection", "ems_profile",
            "ems_profile_read", "ems_set_fmm", "ems_set_precond", "ems_precond_apply",
            "ems_solve_history", "ems_set_progress", "ems_apply_noalloc",
            "ems_set_exponentials")


def lib():
    return _lib


def make_media(host, substrate, omega) -> Media:
    """host/substrate: objects with lam, mu, rho attributes or 3-tuples."""
    def med(m):
        if hasattr(m, "lam"):
            return Medium(m.lam, m.mu, m.rho)
        return Medium(*m)
    return Media(med(host), med(substrate), float(omega))


def smatrix_disk(media: Media, a: float, p: int, bc: int) -> np.ndarray:
    """Closed-form disk scattering matrix [(4p+2), (4p+2)] complex128 (host)."""
    K = 4 * p + 2
    out = np.zeros((K, K), dtype=np.complex128)
    rc = _lib.ems_smatrix_disk(ctypes.byref(media), float(a), int(p), int(bc),
                               out.ctypes.data_as(ctypes.c_void_p))
    if rc != EMS_OK:
        raise EmsError(rc, "ems_smatrix_disk failed")
    return out


def sommerfeld_nodes(media: Media, xy, p, kind=1, q=0, t_max=0.0, delta=0.5, panel_scale=1.0,
                     panel_order=0, tail_factor=0.0, depth_cut=0.0):
    """Host-only node table [q, 6] = (Re xi, Im xi, Re w, Im w, bp, d) and the tail extent."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.int32)
    s = Sommerfeld(int(kind), int(q), float(t_max), float(delta), float(panel_scale), None,
                   int(panel_order), float(tail_factor), float(depth_cut))
    cnt = ctypes.c_int32(0)
    tm = ctypes.c_double(0)
    rc = _lib.ems_sommerfeld_nodes(ctypes.byref(media), ctypes.byref(s), len(p), xy.ctypes.data,
                                   p.ctypes.data, ctypes.byref(cnt), None, ctypes.byref(tm))
    if rc != EMS_OK:
        raise EmsError(rc, "ems_sommerfeld_nodes failed")
    out = np.zeros((cnt.value, 6))
    rc = _lib.ems_sommerfeld_nodes(ctypes.byref(media), ctypes.byref(s), len(p), xy.ctypes.data,
                                   p.ctypes.data, ctypes.byref(cnt), out.ctypes.data, ctypes.byref(tm))
    if rc != EMS_OK:
        raise EmsError(rc, "ems_sommerfeld_nodes failed")
    return out, tm.value


def sommerfeld_depth_cuts(media: Media, xy, p, depth_cut=0.0, **node_opts):
    """Host-only depth truncation of the tabulated Sommerfeld contractions:
    (perm [n], kcut [2, q], ranges [2, n, 2], kept fraction)."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.int32)
    nodes, _ = sommerfeld_nodes(media, xy, p, depth_cut=depth_cut, **node_opts)
    q = nodes.shape[0]
    s = Sommerfeld(int(node_opts.get("kind", 1)), int(node_opts.get("q", 0)),
                   float(node_opts.get("t_max", 0.0)), float(node_opts.get("delta", 0.5)),
                   float(node_opts.get("panel_scale", 1.0)), None,
                   int(node_opts.get("panel_order", 0)), float(node_opts.get("tail_factor", 0.0)),
                   float(depth_cut))
    n = len(p)
    perm = np.zeros(n, dtype=np.int32)
    kcut = np.zeros(2 * q, dtype=np.int32)
    rng = np.zeros(4 * n, dtype=np.int32)
    kept = ctypes.c_double(0.0)
    rc = _lib.ems_sommerfeld_depth_cuts(ctypes.byref(media), ctypes.byref(s), n, xy.ctypes.data,
                                        p.ctypes.data, q, perm.ctypes.data, kcut.ctypes.data,
                                        rng.ctypes.data, ctypes.byref(kept))
    if rc != EMS_OK:
        raise EmsError(rc, "ems_sommerfeld_depth_cuts failed")
    return perm, kcut.reshape(2, q), rng.reshape(2, n, 2), kept.value


def reflection(media: Media, xi: complex) -> np.ndarray:
    """Host-only 2x2 interface reflection R(xi)."""
    out = np.zeros(8)
    rc = _lib.ems_reflection(ctypes.byref(media), float(np.real(xi)), float(np.imag(xi)),
                             out.ctypes.data)
    if rc != EMS_OK:
        raise EmsError(rc, "ems_reflection failed")
    return (out[0::2] + 1j * out[1::2]).reshape(2, 2)


def _stream_ptr(stream=None):
    import torch
    if stream is None and not torch.cuda.is_available():
        return None
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Operator:
    """Handle around one particle cloud, its media, S-matrices and node table."""

    def __init__(self, xy, radius, p, media: Media, S_blocks=None, bc=None, sommerfeld=None,
                 fmm=None):
        self.h = ctypes.c_void_p()
        self._check(_lib.ems_create(ctypes.byref(self.h)))
        self.media = media
        self.n = len(p)
        self.xy = np.ascontiguousarray(xy, dtype=np.float64)
        self.radius = np.ascontiguousarray(radius, dtype=np.float64)
        self.p = np.ascontiguousarray(p, dtype=np.int32)
        self._check(_lib.ems_set_media(self.h, ctypes.byref(media)))
        self._check(_lib.ems_set_particles(self.h, self.n, self.xy.ctypes.data, self.radius.ctypes.data,
                                           self.p.ctypes.data))
        if S_blocks is None:
            if bc is None:
                raise ValueError("give S_blocks or bc for closed-form disks")
            S_blocks = self.disk_blocks(bc)
        self.set_smatrices(S_blocks)
        if sommerfeld is not None:
            self.set_sommerfeld(**sommerfeld)
        if fmm is not None:
            self.set_fmm(**fmm)
        self.built = False

    def set_fmm(self, mode=0, leaf=0, top_boxes=0, digits=0.0):
        """mode 0 automatic, 1 direct sum, 2 FMM."""
        f = Fmm(int(mode), int(leaf), int(top_boxes), float(digits))
        self._check(_lib.ems_set_fmm(self.h, ctypes.byref(f)))
        self.built = False

    def disk_blocks(self, bc):
        cache = {}
        out = []
        for a, pm, b in zip(self.radius, self.p, np.asarray(bc)):
            key = (float(a), int(pm), int(b))
            if key not in cache:
                cache[key] = smatrix_disk(self.media, *key)
            out.append(cache[key])
        return out

    def shape_smatrices(self, kind, a, theta0, bc, npts=0, delta=0.0, stream=None):
        """Scattering matrices of the particles' shapes, generated on the GPU
        (Section 4.3; method of fundamental solutions, ems_smatrix_shapes):
        kind 0 circle, 1 ellipse (semi-axes a, a/2), 2 five-arm star, 3 pear,
        4 starfish (the paper's a1 + a2 cos(a3 t), a2 = a1/4, a3 = 3, 5),
        turned by theta0.  Returns a complex128 device tensor in the packing
        set_smatrices reads (row-major (4p+2)^2 per particle)."""
        import torch
        n = self.n
        kind = np.ascontiguousarray(np.broadcast_to(kind, n), dtype=np.int32)
        a = np.ascontiguousarray(np.broadcast_to(a, n), dtype=np.float64)
        theta0 = np.ascontiguousarray(np.broadcast_to(theta0, n), dtype=np.float64)
        bc = np.ascontiguousarray(np.broadcast_to(bc, n), dtype=np.int32)
        total = int(np.sum((4 * self.p.astype(np.int64) + 2) ** 2))
        out = torch.empty(total, dtype=torch.complex128, device="cuda")
        self._check(_lib.ems_smatrix_shapes(self.h, kind.ctypes.data, a.ctypes.data,
                                            theta0.ctypes.data, bc.ctypes.data, int(npts),
                                            float(delta), ctypes.c_void_p(out.data_ptr()),
                                            _stream_ptr(stream)))
        return out

    def unpack_smatrices(self, flat):
        """Per-particle (4p+2) x (4p+2) blocks (numpy) of a packed S store."""
        flat = flat.cpu().numpy() if hasattr(flat, "cpu") else np.asarray(flat)
        out, o = [], 0
        for pm in self.p:
            K = 4 * int(pm) + 2
            out.append(flat[o: o + K * K].reshape(K, K))
            o += K * K
        return out

    def set_smatrices_rotated(self, prototypes, which, theta0):
        """Per-particle S as turned copies of prototype matrices (Section 4.3):
        S_m = D prototypes[which[m]] D^H, D = diag(e^{-i n theta0[m]})."""
        sizes = [np.asarray(b).size for b in prototypes]
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        flat = np.ascontiguousarray(np.concatenate(
            [np.asarray(b, np.complex128).ravel() for b in prototypes]))
        which = np.ascontiguousarray(np.broadcast_to(which, self.n), dtype=np.int32)
        theta0 = np.ascontiguousarray(np.broadcast_to(theta0, self.n), dtype=np.float64)
        self._check(_lib.ems_set_smatrices_rotated(self.h, len(prototypes), flat.ctypes.data,
                                                   off.ctypes.data, which.ctypes.data,
                                                   theta0.ctypes.data))
        self.built = False

    def set_smatrices_packed(self, flat):
        """S-matrices from one packed array (row-major (4p+2)^2 per particle,
        the output of shape_smatrices; host or device)."""
        flat = flat.cpu().numpy() if hasattr(flat, "cpu") else np.asarray(flat)
        flat = np.ascontiguousarray(flat, dtype=np.complex128)
        sizes = (4 * self.p.astype(np.int64) + 2) ** 2
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        if flat.size != off[-1]:
            raise ValueError("packed S does not match the particles' orders")
        self._S_keep = flat
        self._check(_lib.ems_set_smatrices(self.h, flat.ctypes.data, off.ctypes.data))
        self.built = False

    def set_smatrices(self, blocks):
        sizes = [b.size for b in blocks]
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        flat = np.ascontiguousarray(np.concatenate([np.asarray(b, np.complex128).ravel() for b in blocks]))
        self._S_keep = flat
        self._check(_lib.ems_set_smatrices(self.h, flat.ctypes.data, off.ctypes.data))
        self.built = False

    def set_sommerfeld(self, kind=1, q=0, t_max=0.0, delta=0.5, panel_scale=1.0, nodes=None,
                       panel_order=0, tail_factor=0.0, depth_cut=0.0):
        ptr = None
        if nodes is not None:
            self._nodes_keep = np.ascontiguousarray(nodes, dtype=np.float64)
            ptr = self._nodes_keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            q = self._nodes_keep.shape[0]
        s = Sommerfeld(int(kind), int(q), float(t_max), float(delta), float(panel_scale), ptr,
                       int(panel_order), float(tail_factor), float(depth_cut))
        self._check(_lib.ems_set_sommerfeld(self.h, ctypes.byref(s)))
        self.built = False

    def build(self, stream=None):
        self._check(_lib.ems_build(self.h, _stream_ptr(stream)))
        self.built = True
        return self.info()

    def info(self) -> dict:
        bi = BuildInfo()
        self._check(_lib.ems_get_info(self.h, ctypes.byref(bi)))
        return {k: getattr(bi, k) for k, _ in BuildInfo._fields_}

    @property
    def n_coeff(self) -> int:
        return int(np.sum(2 * (2 * self.p.astype(np.int64) + 1)))

    def _vec_check(self, t, nrhs=None):
        import torch
        if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("coefficient tensors must be contiguous complex128 on the GPU")
        if t.shape[-1] != self.n_coeff:
            raise ValueError(f"last dimension must be n_coeff = {self.n_coeff}")
        return 1 if t.dim() == 1 else t.shape[0]

    def apply(self, x, y=None, flags=EMS_APPLY_ALL, adjoint=False, stream=None):
        import torch
        nrhs = self._vec_check(x)
        if y is None:
            y = torch.empty_like(x)
        self._vec_check(y)
        f = _lib.ems_apply_adjoint if adjoint else _lib.ems_apply
        self._check(f(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), nrhs,
                      int(flags), _stream_ptr(stream)))
        return y

    def apply_noalloc(self, x, y, flags=EMS_APPLY_ALL, stream=None):
        """Forward apply whose workspace is the library's static device array
        (no allocation); y must be preallocated like x."""
        nrhs = self._vec_check(x)
        self._vec_check(y)
        self._check(_lib.ems_apply_noalloc(self.h, ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(y.data_ptr()), nrhs, int(flags),
                                           _stream_ptr(stream)))
        return y

    def incident(self, waves, stream=None):
        """waves: list of (wave, angle); wave 0 = P, 1 = SV from the particle
        side, 2 = P, 3 = SV sent from the substrate."""
        import torch
        arr = (PlaneWave * len(waves))(*[PlaneWave(int(w), float(a)) for w, a in waves])
        out = torch.empty((len(waves), self.n_coeff), dtype=torch.complex128, device="cuda")
        self._check(_lib.ems_incident(self.h, arr, len(waves), ctypes.c_void_p(out.data_ptr()),
                                      _stream_ptr(stream)))
        return out

    def incident_point(self, sources, stream=None):
        """Right-hand sides [nsrc, n_coeff] of point sources in the substrate:
        sources = list of (x0, y0, alpha1, alpha2) with y0 > 0."""
        import torch
        arr = (PointSource * len(sources))(*[PointSource(*map(float, s)) for s in sources])
        out = torch.empty((len(sources), self.n_coeff), dtype=torch.complex128, device="cuda")
        self._check(_lib.ems_incident_point(self.h, arr, len(sources),
                                            ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def background_field_point(self, sources, pts, stream=None):
        """Background displacement [nsrc, npts, 2] of point sources at points of
        either layer (y != 0)."""
        import torch
        arr = (PointSource * len(sources))(*[PointSource(*map(float, s)) for s in sources])
        p = torch.as_tensor(np.ascontiguousarray(pts, dtype=np.float64)).cuda()
        out = torch.empty((len(sources), p.shape[0], 2), dtype=torch.complex128, device="cuda")
        self._check(_lib.ems_eval_background_point(self.h, arr, len(sources), int(p.shape[0]),
                                                   ctypes.c_void_p(p.data_ptr()),
                                                   ctypes.c_void_p(out.data_ptr()),
                                                   _stream_ptr(stream)))
        return out

    def background_field(self, waves, pts, stream=None):
        """Background displacement [nwaves, npts, 2] of plane waves at points of
        either layer (y != 0)."""
        import torch
        arr = (PlaneWave * len(waves))(*[PlaneWave(int(w), float(a)) for w, a in waves])
        p = torch.as_tensor(np.ascontiguousarray(pts, dtype=np.float64)).cuda()
        out = torch.empty((len(waves), p.shape[0], 2), dtype=torch.complex128, device="cuda")
        self._check(_lib.ems_eval_background(self.h, arr, len(waves), int(p.shape[0]),
                                             ctypes.c_void_p(p.data_ptr()),
                                             ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def scattered_field(self, gamma, pts, stream=None):
        """Scattered displacement [nrhs, npts, 2] complex128 at points pts [npts, 2]:
        host points (y < 0) and substrate points (y > 0, transmitted field)."""
        import torch
        nrhs = self._vec_check(gamma)
        p = torch.as_tensor(np.ascontiguousarray(pts, dtype=np.float64)).cuda()
        out = torch.empty((nrhs, p.shape[0], 2), dtype=torch.complex128, device="cuda")
        self._check(_lib.ems_eval_scattered(self.h, ctypes.c_void_p(gamma.data_ptr()), nrhs,
                                            int(p.shape[0]), ctypes.c_void_p(p.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def param_vjp(self, waves, gamma, lam, pts, res, stream=None):
        """(dJ/d centres [n, 2] on the device, (dJ/dlambda_b, dJ/dmu_b)) for the
        misfit residual res = u - u_obs at pts, forward solutions gamma and
        adjoint solutions lam (A^H lam = F^H res)."""
        import torch
        arr = (PlaneWave * len(waves))(*[PlaneWave(int(w), float(a)) for w, a in waves])
        p = torch.as_tensor(np.ascontiguousarray(pts, dtype=np.float64)).cuda()
        res = res.contiguous()
        dxy = torch.empty((self.n, 2), dtype=torch.float64, device="cuda")
        dl = (ctypes.c_double * 2)()
        self._check(_lib.ems_param_vjp(self.h, arr, len(waves), ctypes.c_void_p(gamma.data_ptr()),
                                       ctypes.c_void_p(lam.data_ptr()), int(p.shape[0]),
                                       ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(res.data_ptr()),
                                       ctypes.c_void_p(dxy.data_ptr()), dl, _stream_ptr(stream)))
        return dxy, (dl[0], dl[1])

    def misfit_gradient(self, waves, pts, u_obs, tol=1e-12, restart=200, maxit=2000,
                        precision=0, precond=0):
        """J = 1/2 sum |u - u_obs|^2 over the plane waves and receivers, and its
        gradient: forward solve, field, adjoint right-hand side F^H res,
        adjoint solve, parameter vector-Jacobian product.  u_obs: complex128
        [nwaves, npts, 2] (device or host).  Returns (J, dJ/dxy [n, 2] host,
        (dJ/dlambda_b, dJ/dmu_b), info)."""
        import torch
        b = self.incident(waves)
        gam, i1 = self.solve(b, tol=tol, restart=restart, maxit=maxit, precision=precision,
                             precond=precond)
        if not i1["converged"]:
            raise NotConvergedError("forward", i1)
        u = self.scattered_field(gam, pts)
        res = u - torch.as_tensor(u_obs, dtype=torch.complex128).to(u.device)
        J = 0.5 * float(torch.sum(torch.abs(res) ** 2))
        g = self.scattered_field_adjoint(res, pts)
        lam, i2 = self.solve(g, tol=tol, restart=restart, maxit=maxit, precision=precision,
                             adjoint=True, precond=precond)
        if not i2["converged"]:
            raise NotConvergedError("adjoint", i2)
        dxy, dl = self.param_vjp(waves, gam, lam, pts, res)
        return J, dxy.cpu().numpy(), dl, {"forward": i1, "adjoint": i2}

    def apply_graph(self, x, y, flags=EMS_APPLY_ALL, adjoint=False, stream=None):
        """Apply through a captured HIP graph (captured on the first call with
        these buffers, replayed afterwards).  x, y: complex128 [nrhs, n_coeff]."""
        nrhs = self._vec_check(x)
        self._vec_check(y)
        self._check(_lib.ems_apply_graph(self.h, ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(y.data_ptr()), nrhs, int(flags),
                                         1 if adjoint else 0, _stream_ptr(stream)))
        return y

    def autotune(self, nrhs=1, stream=None) -> dict:
        """Time the matrix-core tile shapes for batches of nrhs; returns the choice."""
        out = (ctypes.c_int32 * 8)()
        self._check(_lib.ems_autotune(self.h, int(nrhs), out, _stream_ptr(stream)))
        v = list(out)
        return {"aggregate_fp64": tuple(v[0:2]), "aggregate_fp32": tuple(v[2:4]),
                "disaggregate_fp64": tuple(v[4:6]), "disaggregate_fp32": tuple(v[6:8])}

    def scattered_field_adjoint(self, res, pts, stream=None):
        """g = F^H res for residuals res [nrhs, npts, 2] at host points pts [npts, 2]."""
        import torch
        res = res.contiguous()
        nrhs = int(res.shape[0])
        p = torch.as_tensor(np.ascontiguousarray(pts, dtype=np.float64)).cuda()
        if tuple(res.shape[1:]) != (p.shape[0], 2) or res.dtype != torch.complex128:
            raise ValueError("res must be complex128 [nrhs, npts, 2]")
        g = torch.empty((nrhs, self.n_coeff), dtype=torch.complex128, device="cuda")
        self._check(_lib.ems_eval_scattered_adjoint(self.h, ctypes.c_void_p(res.data_ptr()), nrhs,
                                                    int(p.shape[0]), ctypes.c_void_p(p.data_ptr()),
                                                    ctypes.c_void_p(g.data_ptr()),
                                                    _stream_ptr(stream)))
        return g

    def solve(self, b, tol=1e-10, restart=200, maxit=1000, precision=0, inner_tol=0.0,
              stream=None, adjoint=False, precond=0, block=False):
        """GMRES on A (or A^H with adjoint=True); precision 1 = mixed iterative
        refinement; precond 1 = cluster block-Jacobi right preconditioner;
        restart 0 = as large as half of the free device memory allows; block =
        one Krylov space per group of up to 64 right-hand sides (FP64; restart
        and maxit then count block steps)."""
        import torch
        nrhs = self._vec_check(b)
        x = torch.empty_like(b)
        o = SolverOpts(float(tol), int(restart), int(maxit), int(precision), float(inner_tol),
                       int(precond), 1 if block else 0)
        info = SolveInfo()
        fn = _lib.ems_solve_adjoint if adjoint else _lib.ems_solve
        rc = fn(self.h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                nrhs, ctypes.byref(o), ctypes.byref(info), _stream_ptr(stream))
        if rc < 0:
            self._check(rc)
        return x, {k: getattr(info, k) for k, _ in SolveInfo._fields_}

    def set_exponentials(self, tabulate=True):
        """Sommerfeld exponentials tabulated at set-up where they fit
        (tabulate=True, the default) or formed in registers by the
        matrix-core kernels (tabulate=False); takes effect at the next build."""
        self._check(_lib.ems_set_exponentials(self.h, 1 if tabulate else 0))

    def set_precond(self, max_unknowns=0):
        """Cluster size of the block-Jacobi preconditioner (unknowns, <= 512)."""
        self._check(_lib.ems_set_precond(self.h, int(max_unknowns)))

    def precond_apply(self, x, adjoint=False, stream=None):
        """(M^{-1} x or M^{-H} x, {clusters, max_rows, setup_s})."""
        import torch
        nrhs = self._vec_check(x)
        y = torch.empty_like(x)
        nc, mr, su = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_double(0.0)
        self._check(_lib.ems_precond_apply(self.h, ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(y.data_ptr()), nrhs,
                                           1 if adjoint else 0, ctypes.byref(nc), ctypes.byref(mr),
                                           ctypes.byref(su), _stream_ptr(stream)))
        return y, {"clusters": nc.value, "max_rows": mr.value, "setup_s": su.value}

    def set_progress(self, fn=None, every=100):
        """fn(iteration, relres) after every ``every`` inner iterations of a
        solve (None switches it off).  The ctypes callback is kept alive on
        the operator."""
        if fn is None:
            self._progress_cb = None
            self._check(_lib.ems_set_progress(self.h, PROGRESS_FN(), 0, None))
            return
        self._progress_cb = PROGRESS_FN(lambda it, rr, _u: fn(int(it), float(rr)))
        self._check(_lib.ems_set_progress(self.h, self._progress_cb, int(every), None))

    def solve_history(self):
        """Estimated relative residual per iteration of the last solve."""
        cnt = ctypes.c_int32(0)
        self._check(_lib.ems_solve_history(self.h, None, 0, ctypes.byref(cnt)))
        out = (ctypes.c_double * max(1, cnt.value))()
        self._check(_lib.ems_solve_history(self.h, out, cnt.value, ctypes.byref(cnt)))
        return np.array(out[:cnt.value])

    def profile(self, enable: bool):
        self._check(_lib.ems_profile(self.h, 1 if enable else 0))

    def profile_read(self) -> dict:
        """{kernel name: (launches, total_ms, algorithmic flops)} from the HIP
        events recorded so far (flops summed over those launches)."""
        arr = (KernelTime * 64)()
        cnt = ctypes.c_int32(0)
        self._check(_lib.ems_profile_read(self.h, arr, 64, ctypes.byref(cnt)))
        return {arr[k].name.decode(): (arr[k].launches, arr[k].total_ms, arr[k].flops)
                for k in range(cnt.value)}

    def _check(self, rc):
        if rc < 0:
            msg = _lib.ems_last_error(self.h).decode() if self.h else ""
            raise EmsError(rc, msg)
        return rc

    def __del__(self):
        try:
            if self.h:
                _lib.ems_destroy(self.h)
                self.h = ctypes.c_void_p()
        except Exception:
            pass


def _autograd_misfit():
    import torch

    class MisfitFunction(torch.autograd.Function):
        """J(xy, lame) = 1/2 sum over plane waves and receivers |u - u_obs|^2.

        Forward builds the operator at the given centres and substrate Lame
        parameters, solves the forward and adjoint systems on the GPU and keeps
        the gradient; backward scales it by the incoming gradient.  Centres
        [n, 2] and lame (lambda_b, mu_b) are float64 tensors."""

        @staticmethod
        def forward(ctx, xy, lame, radius, p, host, substrate_rho, omega, bc, waves, pts,
                    u_obs, S_blocks, sommerfeld, fmm, tol):
            media = make_media(host, (float(lame[0]), float(lame[1]), float(substrate_rho)), omega)
            op = Operator(xy.detach().cpu().numpy(), radius, p, media, S_blocks=S_blocks, bc=bc,
                          sommerfeld=sommerfeld, fmm=fmm)
            op.build()
            J, gxy, gl, _ = op.misfit_gradient(waves, pts, u_obs, tol=tol)
            ctx.save_for_backward(torch.as_tensor(gxy, dtype=torch.float64),
                                  torch.tensor(gl, dtype=torch.float64))
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gout):
            gxy, gl = ctx.saved_tensors
            return (gout * gxy.to(gout.device), gout * gl.to(gout.device)) + (None,) * 13

    return MisfitFunction


def misfit(xy, lame, *, radius, p, host, substrate_rho, omega, waves, pts, u_obs, bc=None,
           S_blocks=None, sommerfeld=None, fmm=None, tol=1e-12):
    """Differentiable receiver misfit (torch.autograd): J as a 0-d tensor whose
    gradient flows to the centres ``xy`` [n, 2] and to ``lame`` = (lambda_b,
    mu_b).  Each call builds the operator at the given parameters."""
    fn = _autograd_misfit()
    return fn.apply(xy, lame, radius, p, host, substrate_rho, omega, bc, waves, pts, u_obs,
                    S_blocks, sommerfeld, fmm, tol)

