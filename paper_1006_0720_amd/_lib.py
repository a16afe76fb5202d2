"""ctypes binding of libpdf.so (the C ABI in include/pdf.h).

Argument marshalling only: every step of the particle method runs in the HIP
kernels of libpdf.so.  PyTorch supplies the device memory (through the
caching allocator hook of pdf_init_mesh) and the HIP stream.  If the library
has not been built this module raises at import: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import weakref
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PDF_LIBRARY") or os.path.join(HERE, "libpdf.so")

PDF_OK = 0
PDF_FP64, PDF_FP32 = 0, 1
FIELD_STATS, FIELD_WP, FIELD_GRADP, FIELD_PRESSURE = 0, 1, 2, 3
NSTAT = 25
NELEMSTAT = 16
NCOUNTERS = 16
COUNTER_NAMES = ["walk_steps", "fallback", "brute", "lost", "reflect", "periodic", "noslip_b",
                 "omega_clamp", "gamma_fail", "empty_node", "nonfinite", "steps", "redist", "ell_iters",
                 "proj_iters", "outflow"]
STATUS = {0: "PDF_OK", 1: "PDF_E_INVALID_ARG", 2: "PDF_E_BAD_MESH", 3: "PDF_E_OOM",
          4: "PDF_E_DEVICE", 5: "PDF_E_STATE", 6: "PDF_E_LOST_PARTICLE", 7: "PDF_E_NUMERIC"}


class PdfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class MeshDesc(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_elems", C.c_int32), ("n_bedges", C.c_int32),
                ("pad", C.c_int32), ("node_xy", C.c_void_p), ("elem_nodes", C.c_void_p),
                ("elem_nbr", C.c_void_p), ("bedge_elem", C.c_void_p), ("bedge_local", C.c_void_p),
                ("bedge_type", C.c_void_p), ("bedge_partner", C.c_void_p),
                ("bedge_shift", C.c_void_p), ("node_master", C.c_void_p)]


class ModelParams(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("model", "wp_source", "omega_source", "tm_mode", "frozen",
                                         "wall_b", "reorder_every", "stats_mode", "min_ppe", "mix_model",
                                         "cond_nu", "cond_nv", "cond_nw", "cond_min", "ell_maxit", "proj",
                                         "proj_maxit", "proj_precond", "ell_precond")] + \
               [(n, C.c_double) for n in ("C0", "C1", "C2", "C3", "C4", "CT", "CL", "Ceta", "Cv",
                                          "gamma5", "Cw1", "Cw2", "Cphi", "nu", "k_floor",
                                          "src_x", "src_y", "src_r", "Cs", "Ct", "nu_wall", "ell_tol", "Cp",
                                          "proj_tol", "inflow_u")]


# fields a parameter set may omit: ELEM statistics, no redistribution, IEM,
# 5 x 5 x 5 conditioning bins with at least 2 particles each, the
# micromixing constants of tab:constants, no wall-function viscosity, the
# conjugate-gradient limits of the elliptic relaxation and of the projection,
# and the multigrid preconditioners of the projection and the elliptic relaxation
PARAM_DEFAULTS = dict(stats_mode=0, min_ppe=0, mix_model=0, cond_nu=5, cond_nv=5, cond_nw=5,
                      cond_min=2, Cs=0.02, Ct=0.7, nu_wall=0.0, ell_maxit=500, ell_tol=1e-12, proj=0,
                      proj_maxit=2000, proj_precond=1, ell_precond=1, Cp=1e-3, proj_tol=1e-12, inflow_u=0.0)


class SeedDesc(C.Structure):
    _fields_ = [("ppe", C.c_int32), ("psi_mode", C.c_int32), ("seed", C.c_uint64),
                ("a", C.c_double), ("b", C.c_double), ("c", C.c_double),
                ("U0", C.c_void_p), ("R0", C.c_void_p), ("Om0", C.c_void_p)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                          "(run __graft_entry__.build() or python -m paper_1006_0720_amd.build)")
    # torch first: it loads the HIP runtime it ships, and the library then
    # binds to that same runtime, the one that owns the memory and streams it
    # is handed.  Loaded first, the library would pull in the system runtime
    # under a name torch's own libraries do not match, torch would load its
    # copy beside it, and the library's first HIP call would fail.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "pdf_init_mesh": ([vp, vp, i32, vp, vp, C.POINTER(vp)], i32),
        "pdf_set_nodal_field": ([vp, i32, vp, i32], i32),
        "pdf_seed_particles": ([vp, vp], i32),
        "pdf_advance": ([vp, i32, dbl], i32),
        "pdf_advance_cfl": ([vp, i32, dbl, dbl, C.POINTER(dbl)], i32),
        "pdf_estimate_stats": ([vp, vp, vp, i32], i32),
        "pdf_get_nodal_field": ([vp, i32, vp, i32], i32),
        "pdf_num_particles": ([vp, C.POINTER(i64)], i32),
        "pdf_get_particles": ([vp, vp, vp, vp], i32),
        "pdf_set_particles": ([vp, i64, vp, vp, vp], i32),
        "pdf_get_counters": ([vp, vp, i32, i32], i32),
        "pdf_enable_timing": ([vp, i32], i32),
        "pdf_get_timing": ([vp, vp, i32], i32),
        "pdf_last_error": ([vp], C.c_char_p),
        "pdf_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


lib = _load()


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Context:
    """One pdf_ctx on one GPU.  mesh: synth.meshes.Mesh-like object with the
    arrays of pdf_mesh_desc; params: dict of pdf_model_params fields."""

    def __init__(self, mesh, params: dict, precision="f64", device=0, stream=None,
                 use_torch_allocator=True, reorder_every=None):
        import torch

        self.torch = torch
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("a ROCm GPU is required (torch.cuda is not available)")
        torch.cuda.set_device(self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.prec = PDF_FP32 if precision == "f32" else PDF_FP64
        self.n_nodes = mesh.n_nodes
        self.n_elems = mesh.n_elems
        self._arrays = [np.ascontiguousarray(mesh.node_xy, np.float64),
                        np.ascontiguousarray(mesh.elem_nodes, np.int32),
                        np.ascontiguousarray(mesh.elem_nbr, np.int32),
                        np.ascontiguousarray(mesh.bedge_elem, np.int32),
                        np.ascontiguousarray(mesh.bedge_local, np.int32),
                        np.ascontiguousarray(mesh.bedge_type, np.int32),
                        np.ascontiguousarray(mesh.bedge_partner, np.int32),
                        np.ascontiguousarray(mesh.bedge_shift, np.float64),
                        np.ascontiguousarray(mesh.node_master, np.int32)]
        a = self._arrays
        md = MeshDesc(mesh.n_nodes, mesh.n_elems, mesh.n_bedges, 0, *[_ptr(x) for x in a])
        mp = ModelParams()
        for name, _ in ModelParams._fields_:
            if name in PARAM_DEFAULTS:
                d = PARAM_DEFAULTS[name]
                setattr(mp, name, type(d)(params.get(name, d)))
                continue
            if name == "reorder_every":
                mp.reorder_every = int(params.get("reorder_every", 0) if reorder_every is None
                                       else reorder_every)
                continue
            setattr(mp, name, params[name])
        self.params = mp
        self._alloc = None
        if use_torch_allocator:
            dev = self.device.index
            strm = self.stream

            def _a(nbytes, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, strm)
                except Exception:
                    return None

            def _f(ptr, user):
                torch.cuda.caching_allocator_delete(ptr)

            self._alloc_fns = (ALLOC_FN(_a), FREE_FN(_f))
            self._alloc = Allocator(self._alloc_fns[0], self._alloc_fns[1], None)
        h = C.c_void_p()
        st = lib.pdf_init_mesh(C.byref(md), C.byref(mp), self.prec,
                               C.byref(self._alloc) if self._alloc is not None else None,
                               C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self.h = h
        if st != PDF_OK:
            msg = lib.pdf_last_error(h).decode() if h.value else ""
            if h.value:
                lib.pdf_destroy(h)
            self.h = None
            raise PdfError(st, msg)

    def _chk(self, st):
        if st != PDF_OK:
            raise PdfError(st, lib.pdf_last_error(self.h).decode())

    def close(self):
        """Destroy the context, after the denoisers made on it (their memory
        comes from the context's allocator and they borrow its mesh)."""
        for dn in list(getattr(self, "_denoisers", ())):
            dn.close()
        if getattr(self, "h", None):
            lib.pdf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- inputs --------------------------------------------------------
    def set_nodal_field(self, field, data):
        if hasattr(data, "data_ptr"):
            t = data.contiguous().to(self.torch.float64)
            self._chk(lib.pdf_set_nodal_field(self.h, field, C.c_void_p(t.data_ptr()), 1))
            self._keep = t
        else:
            arr = np.ascontiguousarray(data, np.float64)
            self._chk(lib.pdf_set_nodal_field(self.h, field, _ptr(arr), 0))

    def seed(self, spec: dict):
        nn = self.n_nodes
        U0 = np.ascontiguousarray(spec["U0"], np.float64).reshape(3, nn)
        R0 = np.ascontiguousarray(spec["R0"], np.float64).reshape(6, nn)
        Om0 = np.ascontiguousarray(spec["Om0"], np.float64).reshape(nn)
        sd = SeedDesc(int(spec["ppe"]), int(spec.get("psi_mode", 0)), int(spec["seed"]),
                      float(spec.get("a", 0.0)), float(spec.get("b", 0.0)), float(spec.get("c", 0.0)),
                      _ptr(U0), _ptr(R0), _ptr(Om0))
        self._chk(lib.pdf_seed_particles(self.h, C.byref(sd)))

    # ---- stepping ------------------------------------------------------
    def advance(self, nsteps, dt):
        self._chk(lib.pdf_advance(self.h, int(nsteps), float(dt)))

    def advance_cfl(self, nsteps, c_cfl, dt_max, wait=True):
        """nsteps steps whose sizes follow eq:CFL (chosen on the device);
        returns the time advanced (waits for the stream), or None with
        wait=False (asynchronous)."""
        t = C.c_double(0.0)
        self._chk(lib.pdf_advance_cfl(self.h, int(nsteps), float(c_cfl), float(dt_max),
                                      C.byref(t) if wait else None))
        return t.value if wait else None

    # ---- outputs -------------------------------------------------------
    def nodal_field(self, field):
        """A nodal field (FIELD_STATS, FIELD_WP or FIELD_GRADP) as (nf, n_nodes)."""
        nf = {FIELD_STATS: NSTAT, FIELD_WP: 9, FIELD_GRADP: 2, FIELD_PRESSURE: 1}[field]
        out = np.empty((nf, self.n_nodes))
        self._chk(lib.pdf_get_nodal_field(self.h, int(field), _ptr(out), 0))
        return out

    def stats(self, elem=False):
        nodal = np.empty((NSTAT, self.n_nodes))
        el = np.empty((NELEMSTAT, self.n_elems)) if elem else None
        self._chk(lib.pdf_estimate_stats(self.h, _ptr(nodal), _ptr(el), 0))
        return (nodal, el) if elem else nodal

    def stats_device(self):
        """Nodal statistics copied into a new torch tensor on the context's device."""
        t = self.torch.empty((NSTAT, self.n_nodes), dtype=self.torch.float64, device=self.device)
        self._chk(lib.pdf_estimate_stats(self.h, C.c_void_p(t.data_ptr()), None, 1))
        return t

    def num_particles(self):
        n = C.c_int64()
        self._chk(lib.pdf_num_particles(self.h, C.byref(n)))
        return n.value

    def particles(self, sort_by_id=True):
        n = self.num_particles()
        state = np.empty((7, n))
        elem = np.empty(n, np.int32)
        pid = np.empty(n, np.uint32)
        self._chk(lib.pdf_get_particles(self.h, _ptr(state), _ptr(elem), _ptr(pid)))
        if sort_by_id:
            o = np.argsort(pid, kind="stable")
            return state[:, o], elem[o], pid[o]
        return state, elem, pid

    def set_particles(self, state, elem, pid):
        state = np.ascontiguousarray(state, np.float64)
        elem = np.ascontiguousarray(elem, np.int32)
        pid = np.ascontiguousarray(pid, np.uint32)
        self._chk(lib.pdf_set_particles(self.h, state.shape[1], _ptr(state), _ptr(elem), _ptr(pid)))

    def counters(self, reset=False):
        out = np.zeros(NCOUNTERS, np.uint64)
        self._chk(lib.pdf_get_counters(self.h, _ptr(out), NCOUNTERS, int(reset)))
        return {n: int(v) for n, v in zip(COUNTER_NAMES, out)}

    def enable_timing(self, on=True):
        self._chk(lib.pdf_enable_timing(self.h, int(on)))

    def timing(self):
        out = np.zeros(5)
        self._chk(lib.pdf_get_timing(self.h, _ptr(out), 5))
        return dict(elem_prep=out[0], advance=out[1], estimator=out[2], reorder=out[3], step_start=out[4])


def _declare_denoiser():
    vp, i32, i64, dbl, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint64
    sig = {
        "pdf_denoiser_create": ([vp, i32, u64, C.POINTER(vp)], i32),
        "pdf_denoiser_destroy": ([vp], None),
        "pdf_denoiser_params": ([vp, vp, i64, i32], i32),
        "pdf_denoiser_set_norm": ([vp, vp, vp, vp], i32),
        "pdf_denoiser_set_fallback": ([vp, vp], i32),
        "pdf_denoiser_io": ([vp, i32, C.c_char_p], i32),
        "pdf_denoiser_features": ([vp, vp, vp, i32], i32),
        "pdf_denoiser_forward": ([vp, vp, i32, vp], i32),
        "pdf_denoiser_train_step": ([vp, vp, vp, i32, C.c_float, C.POINTER(C.c_float), vp], i32),
        "pdf_denoise_stats": ([vp, dbl, vp, i32, C.POINTER(u64)], i32),
        "pdf_denoise_stats_noalloc": ([vp, dbl, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res


_declare_denoiser()

DN_NIN, DN_NOUT = 48, 8


def dn_nparam(h):
    return 48 * h + h + 2 * (h * h + h) + h * 8 + 8


class Denoiser:
    """Learned denoiser bound to a Context (its mesh and latest statistics).
    Device arrays are torch tensors on the context's device."""

    def __init__(self, ctx: Context, hidden=128, seed=0):
        self.ctx = ctx
        self.torch = ctx.torch
        self.hidden = hidden
        self.n_param = dn_nparam(hidden)
        h = C.c_void_p()
        ctx._chk(lib.pdf_denoiser_create(ctx.h, hidden, seed, C.byref(h)))
        self.h = h
        if not hasattr(ctx, "_denoisers"):
            ctx._denoisers = weakref.WeakSet()
        ctx._denoisers.add(self)

    def close(self):
        # a denoiser whose context is already gone was destroyed with it
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            lib.pdf_denoiser_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        out = np.empty(self.n_param, np.float32)
        self.ctx._chk(lib.pdf_denoiser_params(self.h, _ptr(out), self.n_param, 0))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        assert p.size == self.n_param
        self.ctx._chk(lib.pdf_denoiser_params(self.h, _ptr(p), self.n_param, 1))

    def set_norm(self, mu, sig, scale):
        mu, sig, scale = (np.ascontiguousarray(a, np.float32) for a in (mu, sig, scale))
        self.ctx._chk(lib.pdf_denoiser_set_norm(self.h, _ptr(mu), _ptr(sig), _ptr(scale)))
        self.norm = (mu.copy(), sig.copy(), scale.copy())

    def set_fallback(self, kappa):
        """Per-statistic calibration of the fallback test (8 positive factors)."""
        kappa = np.ascontiguousarray(kappa, np.float32)
        assert kappa.size == DN_NOUT
        self.ctx._chk(lib.pdf_denoiser_set_fallback(self.h, _ptr(kappa)))
        self.kappa = kappa.copy()

    def save(self, path):
        """pdf_denoiser_io: write the parameters, standardisation, output
        scales and fallback factors to path."""
        self.ctx._chk(lib.pdf_denoiser_io(self.h, 1, os.fsencode(path)))

    def load(self, path):
        """pdf_denoiser_io: read a file written by save() (same hidden width).
        The host copies of the standardisation and fallback factors that
        set_norm and set_fallback keep are then unknown (None)."""
        self.ctx._chk(lib.pdf_denoiser_io(self.h, 0, os.fsencode(path)))
        self.norm = None
        self.kappa = None

    def features(self, nodal=None, standardized=False):
        """Features [n_nodes, 48] (torch, device) of nodal statistics (torch
        device tensor [25, n_nodes] or None for the latest estimate)."""
        t = self.torch
        out = t.empty((self.ctx.n_nodes, DN_NIN), dtype=t.float32, device=self.ctx.device)
        src = None if nodal is None else C.c_void_p(nodal.contiguous().data_ptr())
        self.ctx._chk(lib.pdf_denoiser_features(self.h, src, C.c_void_p(out.data_ptr()), int(standardized)))
        return out

    def forward(self, x):
        t = self.torch
        x = x.contiguous().to(t.float32)
        y = t.empty((x.shape[0], DN_NOUT), dtype=t.float32, device=self.ctx.device)
        self.ctx._chk(lib.pdf_denoiser_forward(self.h, C.c_void_p(x.data_ptr()), x.shape[0],
                                               C.c_void_p(y.data_ptr())))
        return y

    def train_step(self, x, target, lr, want_grad=False):
        t = self.torch
        x = x.contiguous().to(t.float32)
        target = target.contiguous().to(t.float32)
        loss = C.c_float()
        g = np.empty(self.n_param, np.float32) if want_grad else None
        self.ctx._chk(lib.pdf_denoiser_train_step(self.h, C.c_void_p(x.data_ptr()),
                                                  C.c_void_p(target.data_ptr()), x.shape[0],
                                                  float(lr), C.byref(loss), _ptr(g)))
        return (loss.value, g) if want_grad else loss.value

    def denoise(self, tau=3.0, device=False):
        """Denoised copy of the latest nodal statistics and the number of
        rejected corrections; a numpy array, or a torch device tensor if device."""
        nf = C.c_uint64()
        if device:
            out = self.torch.empty((NSTAT, self.ctx.n_nodes), dtype=self.torch.float64,
                                   device=self.ctx.device)
            self.ctx._chk(lib.pdf_denoise_stats(self.h, float(tau), C.c_void_p(out.data_ptr()), 1,
                                                C.byref(nf)))
        else:
            out = np.empty((NSTAT, self.ctx.n_nodes))
            self.ctx._chk(lib.pdf_denoise_stats(self.h, float(tau), _ptr(out), 0, C.byref(nf)))
        return out, nf.value

    def denoise_into(self, out, tau=3.0):
        """pdf_denoise_stats into a caller-owned device tensor (float64
        [25, n_nodes]) without the rejection count: queued on the context's
        stream, the call does not wait for it."""
        t = self.torch
        assert out.dtype == t.float64 and out.is_contiguous() and tuple(out.shape) == (NSTAT, self.ctx.n_nodes)
        self.ctx._chk(lib.pdf_denoise_stats(self.h, float(tau), C.c_void_p(out.data_ptr()), 1, None))
        return out

    def denoise_noalloc(self, out, n_fallback=None, tau=3.0):
        """pdf_denoise_stats_noalloc into caller-owned device tensors: out
        (float64 [25, n_nodes]) and n_fallback (int64 [1] or None)."""
        t = self.torch
        assert out.dtype == t.float64 and out.is_contiguous() and tuple(out.shape) == (NSTAT, self.ctx.n_nodes)
        nfp = None
        if n_fallback is not None:
            assert n_fallback.dtype == t.int64 and n_fallback.numel() >= 1
            nfp = C.c_void_p(n_fallback.data_ptr())
        self.ctx._chk(lib.pdf_denoise_stats_noalloc(self.h, float(tau), C.c_void_p(out.data_ptr()), nfp))
