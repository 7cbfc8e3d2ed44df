"""Python binding of liblp (include/lp.h): argument marshalling only.

Every step of the method runs in the HIP kernels of ``liblp.so``; this module
passes device pointers of torch tensors and the current HIP stream.  It raises
if the library has not been built -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblp.so")

OK, E_ARG, E_CAPACITY, E_NUMERIC, E_DEVICE, E_NOMEM, E_STATE = range(7)
FP64, MIXED = 0, 1
EST_PLAIN, EST_INJECTED, EST_MLP = 0, 1, 2
FLAG_LIMITED, FLAG_DEGENERATE, FLAG_VACUUM, FLAG_SUBSTITUTED, FLAG_FALLBACK, FLAG_NUMERIC = 1, 2, 4, 8, 16, 32

EXPORTS = ["lp_config_default", "lp_create", "lp_destroy", "lp_workspace_bytes", "lp_set_workspace", "lp_neighbors",
           "lp_neighbors_noalloc", "lp_gfd", "lp_gfd3", "lp_outflow",
           "lp_reservoir_inflow", "lp_inflow_layer", "lp_step", "lp_run", "lp_run_open",
           "lp_conservation", "lp_check", "lp_get_info", "lp_set_time", "lp_profile", "lp_profile_read",
           "lp_set_tuning", "lp_get_tuning", "lp_autotune", "lp_train_cfg_default", "lp_features", "lp_mlp_init",
           "lp_mlp_set", "lp_mlp_get", "lp_mlp_forward", "lp_mlp_grad", "lp_mlp_train", "lp_status_str",
           "lp_last_error"]
MLP_NPARAM = 5313
MLP_NIN = 16
(TUNE_SEARCH_MODE, TUNE_SEARCH_GROUP, TUNE_SOLVE_BLOCK, TUNE_SOLVE_MODE, TUNE_QUEUE_TILE, TUNE_SEARCH_CAP,
 TUNE_LIST_SKIN) = range(7)
TUNE_COUNT = 7
TUNE_NAMES = ["search_mode", "search_group", "solve_block", "solve_mode", "queue_tile", "search_cap", "list_skin"]
STAGES = ["prep", "cells", "search", "fit", "update", "fallback", "step", "mlp"]


class LpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("liblp status %d: %s" % (status, msg))
        self.status = status


class Config(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("precision", C.c_int32), ("estimator", C.c_int32), ("max_nb", C.c_int32),
        ("lw_cap", C.c_int32), ("uw_cap", C.c_int32), ("refine", C.c_int32), ("vacuum", C.c_int32),
        ("gamma", C.c_double), ("cfl", C.c_double), ("kappa", C.c_double), ("est_eps", C.c_double),
        ("cond_max", C.c_double), ("uw_cond_max", C.c_double), ("cond_fallback", C.c_double),
        ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
        ("periodic_mask", C.c_uint32), ("wall_lo_mask", C.c_uint32), ("wall_hi_mask", C.c_uint32),
        ("mlp_band", C.c_float), ("mlp_feat_max", C.c_float), ("refine_cond", C.c_float),
        ("limiter_cap", C.c_float), ("reserved", C.c_int32 * 5),
    ]


class TrainCfg(C.Structure):
    _fields_ = [
        ("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
        ("eps", C.c_float), ("seed", C.c_uint64), ("reserved", C.c_int32 * 6),
    ]


class Particles(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("x", C.c_void_p * 3), ("V", C.c_void_p), ("u", C.c_void_p * 3), ("P", C.c_void_p),
        ("m", C.c_void_p), ("phi", C.c_void_p), ("flags", C.c_void_p),
    ]


class Info(C.Structure):
    _fields_ = [
        ("t", C.c_double), ("dt", C.c_double), ("n_ghost", C.c_int64), ("max_count", C.c_int32),
        ("n_fallback", C.c_int32), ("n_limited", C.c_int64), ("error_bits", C.c_uint32), ("levels", C.c_int32 * 2),
        ("n_mlp", C.c_int64), ("n_mlp_plain", C.c_int64), ("n_refined", C.c_int64), ("n_list_builds", C.c_int64),
        ("n_captures", C.c_int64),
    ]


class OpenBC(C.Structure):
    _fields_ = [
        ("out_lo_mask", C.c_uint32), ("out_hi_mask", C.c_uint32), ("in_every", C.c_int32), ("in_axis", C.c_int32),
        ("in_side", C.c_int32), ("spacing", C.c_double), ("depth", C.c_double), ("rho", C.c_double),
        ("p_in", C.c_double), ("u_n", C.c_double), ("res_width", C.c_double), ("res_p", C.c_double),
        ("res_rho", C.c_double),
    ]


_lib = None


def lib():
    """Load liblp.so (built by ``python -m paper_2206_11998_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblp.so is not built; run `python -m paper_2206_11998_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.lp_config_default.restype = None
        L.lp_config_default.argtypes = [C.POINTER(Config), i32]
        L.lp_create.restype = i32
        L.lp_create.argtypes = [C.POINTER(Config), C.POINTER(vp)]
        L.lp_destroy.restype = i32
        L.lp_destroy.argtypes = [vp]
        L.lp_neighbors.restype = i32
        L.lp_neighbors.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp]
        L.lp_workspace_bytes.restype = i32
        L.lp_workspace_bytes.argtypes = [vp, vp, C.POINTER(Particles), C.POINTER(C.c_int64)]
        L.lp_set_workspace.restype = i32
        L.lp_set_workspace.argtypes = [vp, vp, vp, i64]
        L.lp_neighbors_noalloc.restype = i32
        L.lp_neighbors_noalloc.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp]
        L.lp_gfd.restype = i32
        L.lp_gfd.argtypes = [vp, vp, i64, vp, vp, vp, vp, i32, C.POINTER(vp), vp, vp]
        L.lp_outflow.restype = i32
        L.lp_outflow.argtypes = [vp, vp, C.c_void_p, C.c_uint32, C.c_uint32, C.POINTER(C.c_int64)]
        L.lp_reservoir_inflow.restype = i32
        L.lp_reservoir_inflow.argtypes = [vp, vp, C.c_void_p, i32, i32, C.c_double, C.c_double, C.c_double,
                                          C.POINTER(C.c_double)]
        L.lp_inflow_layer.restype = i32
        L.lp_inflow_layer.argtypes = [vp, vp, C.c_void_p, i64, i32, i32, C.c_double, C.c_double, C.c_double,
                                      C.c_double, C.c_double, C.POINTER(C.c_int64)]
        L.lp_gfd3.restype = i32
        L.lp_gfd3.argtypes = [vp, vp, i64, vp, vp, vp, vp, i32, C.POINTER(vp), vp, vp]
        L.lp_step.restype = i32
        L.lp_step.argtypes = [vp, vp, C.POINTER(Particles), dbl]
        L.lp_run.restype = i32
        L.lp_run.argtypes = [vp, vp, C.POINTER(Particles), i32, dbl]
        L.lp_run_open.restype = i32
        L.lp_run_open.argtypes = [vp, vp, C.POINTER(Particles), i64, C.POINTER(OpenBC), i32, dbl,
                                  C.POINTER(C.c_int64)]
        L.lp_conservation.restype = i32
        L.lp_conservation.argtypes = [vp, vp, C.POINTER(Particles), C.POINTER(C.c_double)]
        L.lp_check.restype = i32
        L.lp_check.argtypes = [vp, vp]
        L.lp_get_info.restype = i32
        L.lp_get_info.argtypes = [vp, vp, C.POINTER(Info)]
        L.lp_set_time.restype = i32
        L.lp_set_time.argtypes = [vp, vp, dbl]
        L.lp_profile.restype = i32
        L.lp_profile.argtypes = [vp, i32]
        L.lp_profile_read.restype = i32
        L.lp_profile_read.argtypes = [vp, vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.lp_set_tuning.restype = i32
        L.lp_set_tuning.argtypes = [vp, i32, i32]
        L.lp_get_tuning.restype = i32
        L.lp_get_tuning.argtypes = [vp, i32, C.POINTER(i32)]
        L.lp_autotune.restype = i32
        L.lp_autotune.argtypes = [vp, vp, C.POINTER(Particles), i32, C.POINTER(i32), C.POINTER(C.c_double)]
        fp = C.POINTER(C.c_float)
        L.lp_train_cfg_default.restype = None
        L.lp_train_cfg_default.argtypes = [C.POINTER(TrainCfg)]
        L.lp_features.restype = i32
        L.lp_features.argtypes = [vp, vp, C.POINTER(Particles), vp, vp, vp]
        L.lp_mlp_init.restype = i32
        L.lp_mlp_init.argtypes = [vp, C.c_uint64]
        L.lp_mlp_set.restype = i32
        L.lp_mlp_set.argtypes = [vp, fp, i64]
        L.lp_mlp_get.restype = i32
        L.lp_mlp_get.argtypes = [vp, fp, i64]
        L.lp_mlp_forward.restype = i32
        L.lp_mlp_forward.argtypes = [vp, vp, i64, vp, vp, vp]
        L.lp_mlp_grad.restype = i32
        L.lp_mlp_grad.argtypes = [vp, vp, i64, vp, vp, fp, fp]
        L.lp_mlp_train.restype = i32
        L.lp_mlp_train.argtypes = [vp, vp, i64, vp, vp, C.POINTER(TrainCfg), fp]
        L.lp_status_str.restype = C.c_char_p
        L.lp_status_str.argtypes = [i32]
        L.lp_last_error.restype = C.c_char_p
        L.lp_last_error.argtypes = [vp]
        _lib = L
    return _lib


def make_config(cfg: dict, precision: str = "fp64", estimator: str = "plain", refine: bool = True,
                refine_cond: float = 0.0) -> Config:
    """lp_config from a workload config dict (see workloads.base_config).
    refine_cond > 0 refines only the mixed fits whose condition estimate
    exceeds it (0: every fit)."""
    c = Config()
    d = int(cfg["dim"])
    lib().lp_config_default(C.byref(c), d)
    c.precision = {"fp64": FP64, "mixed": MIXED}[precision]
    c.estimator = {"plain": EST_PLAIN, "injected": EST_INJECTED, "mlp": EST_MLP}[estimator]
    c.refine = int(bool(refine))
    c.refine_cond = float(refine_cond)
    c.max_nb = int(cfg.get("max_nb", 128))
    c.lw_cap = int(cfg.get("lw_cap", 0))
    c.uw_cap = int(cfg.get("uw_cap", 0))
    c.vacuum = int(bool(cfg.get("vacuum", False)))
    c.gamma = float(cfg.get("gamma", 1.4))
    c.cfl = float(cfg.get("cfl", 0.5))
    c.kappa = float(cfg["kappa"])
    c.est_eps = float(cfg.get("est_eps", 1e-5))
    c.cond_max = float(cfg.get("cond_max", 1e12))
    c.uw_cond_max = float(cfg.get("uw_cond_max", 1e2))
    c.cond_fallback = float(cfg.get("cond_fallback", 1e6))
    c.limiter_cap = float(cfg.get("limiter_cap", 1.0))
    for a in range(3):
        c.box_lo[a] = float(cfg["box_lo"][a]) if a < d else 0.0
        c.box_hi[a] = float(cfg["box_hi"][a]) if a < d else 1.0
    c.periodic_mask = sum(1 << a for a in range(d) if cfg["periodic"][a])
    c.wall_lo_mask = sum(1 << a for a in range(d) if cfg.get("wall_lo", [False] * d)[a])
    c.wall_hi_mask = sum(1 << a for a in range(d) if cfg.get("wall_hi", [False] * d)[a])
    return c


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def state_to_device(state: dict, device="cuda"):
    """numpy workload state -> dict of contiguous torch tensors on the GPU (SoA)."""
    import torch
    d = state["x"].shape[1]
    out = {
        "x": [torch.from_numpy(np.ascontiguousarray(state["x"][:, a])).to(device) for a in range(d)],
        "u": [torch.from_numpy(np.ascontiguousarray(state["u"][:, a])).to(device) for a in range(d)],
        "V": torch.from_numpy(np.ascontiguousarray(state["V"])).to(device),
        "P": torch.from_numpy(np.ascontiguousarray(state["P"])).to(device),
        "m": torch.from_numpy(np.ascontiguousarray(state["m"])).to(device),
    }
    n = out["V"].shape[0]
    out["phi"] = torch.zeros(n, dtype=torch.float32, device=device)
    out["flags"] = torch.zeros(n, dtype=torch.uint8, device=device)
    return out


def state_to_host(st: dict) -> dict:
    """Device state -> numpy dict in the workload layout."""
    return {
        "x": np.stack([t.cpu().numpy() for t in st["x"]], axis=1),
        "u": np.stack([t.cpu().numpy() for t in st["u"]], axis=1),
        "V": st["V"].cpu().numpy(), "P": st["P"].cpu().numpy(), "m": st["m"].cpu().numpy(),
        "phi": st["phi"].cpu().numpy(), "flags": st["flags"].cpu().numpy(),
    }


class Context:
    """One liblp context (one per stream)."""

    def __init__(self, cfg: dict, precision="fp64", estimator="plain", refine=True, refine_cond=0.0):
        self.cfg = cfg
        self.dim = int(cfg["dim"])
        self.max_nb = int(cfg.get("max_nb", 128))
        self._c = make_config(cfg, precision, estimator, refine, refine_cond)
        h = C.c_void_p()
        st = lib().lp_create(C.byref(self._c), C.byref(h))
        if st != OK:
            raise LpError(st, "lp_create failed (see stderr)")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().lp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st):
        if st != OK:
            raise LpError(st, lib().lp_last_error(self._h).decode())

    def _particles(self, s: dict) -> Particles:
        p = Particles()
        p.n = s["V"].shape[0]
        for a in range(3):
            p.x[a] = s["x"][a].data_ptr() if a < self.dim else None
            p.u[a] = s["u"][a].data_ptr() if a < self.dim else None
        p.V = s["V"].data_ptr()
        p.P = s["P"].data_ptr()
        p.m = s["m"].data_ptr()
        p.phi = s["phi"].data_ptr() if s.get("phi") is not None else None
        p.flags = s["flags"].data_ptr() if s.get("flags") is not None else None
        self._keep = s
        return p

    def neighbors(self, x, r, stream=None):
        """x: list of D float64 CUDA tensors; r: float64 CUDA tensor -> (count, idx[n, max_nb])."""
        import torch
        n = r.shape[0]
        count = torch.empty(n, dtype=torch.int32, device=r.device)
        idx = torch.full((n, self.max_nb), -1, dtype=torch.int32, device=r.device)
        z = x[2] if self.dim == 3 else None
        st = lib().lp_neighbors(self._h, _stream_ptr(stream), n, _ptr(x[0]), _ptr(x[1]), _ptr(z), _ptr(r),
                                _ptr(count), _ptr(idx))
        if st not in (OK, E_CAPACITY):
            self._raise(st)
        return count, idx, st

    def workspace_bytes(self, s: dict, stream=None) -> int:
        """lp_workspace_bytes: device bytes a step of these particles needs in a caller block."""
        p = self._particles(s)
        b = C.c_int64(0)
        self._raise(lib().lp_workspace_bytes(self._h, _stream_ptr(stream), C.byref(p), C.byref(b)))
        return b.value

    def set_workspace(self, buf, stream=None):
        """lp_set_workspace over a CUDA uint8 tensor (kept alive here); None: library-allocated buffers."""
        if buf is None:
            self._ws = None
            self._raise(lib().lp_set_workspace(self._h, _stream_ptr(stream), None, 0))
            return
        self._ws = buf
        self._raise(lib().lp_set_workspace(self._h, _stream_ptr(stream), C.c_void_p(buf.data_ptr()),
                                           int(buf.numel() * buf.element_size())))

    def neighbors_noalloc(self, x, r, count, idx, stream=None):
        """lp_neighbors_noalloc into the caller's count[n] / idx[n, max_nb]
        (int32 CUDA tensors); returns the status."""
        n = r.shape[0]
        z = x[2] if self.dim == 3 else None
        return lib().lp_neighbors_noalloc(self._h, _stream_ptr(stream), n, _ptr(x[0]), _ptr(x[1]), _ptr(z), _ptr(r),
                                          _ptr(count), _ptr(idx))

    def gfd(self, x, r, fields, stream=None):
        """Second-order GFD derivatives: deriv[f, c, i], status[i]."""
        import torch
        n = r.shape[0]
        nu = 9 if self.dim == 3 else 5
        nf = len(fields)
        deriv = torch.zeros((nf, nu, n), dtype=torch.float64, device=r.device)
        status = torch.zeros(n, dtype=torch.uint8, device=r.device)
        fp = (C.c_void_p * nf)(*[f.data_ptr() for f in fields])
        z = x[2] if self.dim == 3 else None
        st = lib().lp_gfd(self._h, _stream_ptr(stream), n, _ptr(x[0]), _ptr(x[1]), _ptr(z), _ptr(r), nf, fp,
                          _ptr(deriv), _ptr(status))
        self._raise(st)
        return deriv, status

    def gfd3(self, x, r, fields, stream=None):
        """Third-order GFD derivatives: deriv[f, c, i] over the 19 (3D) / 9 (2D)
        columns of lp_gfd3, status[i]."""
        import torch
        n = r.shape[0]
        nu = 19 if self.dim == 3 else 9
        nf = len(fields)
        deriv = torch.zeros((nf, nu, n), dtype=torch.float64, device=r.device)
        status = torch.zeros(n, dtype=torch.uint8, device=r.device)
        fp = (C.c_void_p * nf)(*[f.data_ptr() for f in fields])
        z = x[2] if self.dim == 3 else None
        st = lib().lp_gfd3(self._h, _stream_ptr(stream), n, _ptr(x[0]), _ptr(x[1]), _ptr(z), _ptr(r), nf, fp,
                           _ptr(deriv), _ptr(status))
        self._raise(st)
        return deriv, status

    def outflow(self, s: dict, lo_mask: int, hi_mask: int, stream=None) -> int:
        """Delete the particles past the outflow faces, in place; returns the
        number kept (the first that many entries of every array)."""
        p = self._particles(s)
        kept = C.c_int64(0)
        self._raise(lib().lp_outflow(self._h, _stream_ptr(stream), C.byref(p), int(lo_mask), int(hi_mask),
                                     C.byref(kept)))
        return kept.value

    def reservoir_inflow(self, s: dict, axis: int, side: int, width: float, p_res: float, rho_res: float,
                         stream=None):
        """(P_in, rho_in, u_in, particles averaged) of the reservoir inflow condition."""
        p = self._particles(s)
        out = (C.c_double * 4)()
        self._raise(lib().lp_reservoir_inflow(self._h, _stream_ptr(stream), C.byref(p), int(axis), int(side),
                                              float(width), float(p_res), float(rho_res), out))
        return np.array(out[:])

    def inflow_layer(self, s: dict, n: int, axis: int, side: int, spacing: float, depth: float, rho: float,
                     p_in: float, u_n: float, stream=None) -> int:
        """Append one lattice layer of inflow particles after the first n
        entries of s (whose arrays are the capacity); returns the new count."""
        p = self._particles(s)
        cap = p.n
        p.n = int(n)
        n_new = C.c_int64(0)
        self._raise(lib().lp_inflow_layer(self._h, _stream_ptr(stream), C.byref(p), cap, int(axis), int(side),
                                          float(spacing), float(depth), float(rho), float(p_in), float(u_n),
                                          C.byref(n_new)))
        return n_new.value

    def step(self, s: dict, dt: float = 0.0, stream=None):
        p = self._particles(s)
        self._raise(lib().lp_step(self._h, _stream_ptr(stream), C.byref(p), float(dt)))

    def run(self, s: dict, nsteps: int, t_end: float = 0.0, stream=None):
        p = self._particles(s)
        self._raise(lib().lp_run(self._h, _stream_ptr(stream), C.byref(p), int(nsteps), float(t_end)))

    def run_open(self, s: dict, n: int, nsteps: int, t_end: float = 0.0, out_lo_mask: int = 0, out_hi_mask: int = 0,
                 in_every: int = 0, in_axis: int = 0, in_side: int = 0, spacing: float = 0.0, depth: float = 0.0,
                 rho: float = 0.0, p_in: float = 0.0, u_n: float = 0.0, res_width: float = 0.0, res_p: float = 0.0,
                 res_rho: float = 0.0, stream=None) -> int:
        """lp_run with outflow faces and a periodic inflow layer inside the
        steps; the first n entries of s are the particles, its arrays the
        capacity.  Returns the count after the run (the arrays compacted)."""
        p = self._particles(s)
        cap = p.n
        p.n = int(n)
        bc = OpenBC(int(out_lo_mask), int(out_hi_mask), int(in_every), int(in_axis), int(in_side), float(spacing),
                    float(depth), float(rho), float(p_in), float(u_n), float(res_width), float(res_p),
                    float(res_rho))
        n_out = C.c_int64(0)
        self._raise(lib().lp_run_open(self._h, _stream_ptr(stream), C.byref(p), cap, C.byref(bc), int(nsteps),
                                      float(t_end), C.byref(n_out)))
        return n_out.value

    def conservation(self, s: dict, stream=None):
        p = self._particles(s)
        out = (C.c_double * 5)()
        self._raise(lib().lp_conservation(self._h, _stream_ptr(stream), C.byref(p), out))
        return np.array(out[:])

    def check(self, stream=None):
        return lib().lp_check(self._h, _stream_ptr(stream))

    def info(self, stream=None) -> dict:
        inf = Info()
        self._raise(lib().lp_get_info(self._h, _stream_ptr(stream), C.byref(inf)))
        return {"t": inf.t, "dt": inf.dt, "n_ghost": inf.n_ghost, "max_count": inf.max_count,
                "n_fallback": inf.n_fallback, "n_limited": inf.n_limited, "error_bits": inf.error_bits,
                "levels": (inf.levels[0], inf.levels[1]), "n_mlp": inf.n_mlp, "n_mlp_plain": inf.n_mlp_plain,
                "n_refined": inf.n_refined, "n_list_builds": inf.n_list_builds, "n_captures": inf.n_captures}

    def set_time(self, t: float, stream=None):
        self._raise(lib().lp_set_time(self._h, _stream_ptr(stream), float(t)))

    def profile(self, enable: bool):
        self._raise(lib().lp_profile(self._h, int(bool(enable))))

    def profile_read(self, stream=None) -> dict:
        """Per-stage summed milliseconds and launch counts since profiling started."""
        ms = (C.c_double * len(STAGES))()
        cnt = (C.c_int64 * len(STAGES))()
        self._raise(lib().lp_profile_read(self._h, _stream_ptr(stream), ms, cnt))
        return {name: (ms[q], cnt[q]) for q, name in enumerate(STAGES)}

    def set_tuning(self, param: int, value: int):
        self._raise(lib().lp_set_tuning(self._h, int(param), int(value)))

    def get_tuning(self, param: int) -> int:
        v = C.c_int32(0)
        self._raise(lib().lp_get_tuning(self._h, int(param), C.byref(v)))
        return v.value

    def autotune(self, s: dict, reps: int = 3, stream=None):
        """Choose the launch shapes by timing steps of a private copy of s
        (s is not modified).  Returns ({name: value}, ms per step)."""
        p = self._particles(s)
        best = (C.c_int32 * TUNE_COUNT)()
        ms = C.c_double(0.0)
        self._raise(lib().lp_autotune(self._h, _stream_ptr(stream), C.byref(p), int(reps), best, C.byref(ms)))
        return {name: best[q] for q, name in enumerate(TUNE_NAMES)}, ms.value


def train_cfg(**kw) -> TrainCfg:
    """lp_train_cfg with the library defaults, overridden by keyword."""
    t = TrainCfg()
    lib().lp_train_cfg_default(C.byref(t))
    for k, v in kw.items():
        setattr(t, k, v)
    return t


def _ctx_features(self, s: dict, stream=None):
    """Network inputs (n x 16 float32), quotient-estimator phi (n) and
    validity (n, uint8) of every particle of s at its current state."""
    import torch
    p = self._particles(s)
    n = s["V"].shape[0]
    dev = s["V"].device
    feat = torch.empty((n, MLP_NIN), dtype=torch.float32, device=dev)
    phi = torch.empty(n, dtype=torch.float32, device=dev)
    valid = torch.empty(n, dtype=torch.uint8, device=dev)
    self._raise(lib().lp_features(self._h, _stream_ptr(stream), C.byref(p), _ptr(feat), _ptr(phi), _ptr(valid)))
    return feat, phi, valid


def _ctx_mlp_init(self, seed: int = 1):
    self._raise(lib().lp_mlp_init(self._h, int(seed)))


def _ctx_mlp_set(self, params):
    a = np.ascontiguousarray(params, dtype=np.float32)
    self._raise(lib().lp_mlp_set(self._h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))


def _ctx_mlp_get(self) -> np.ndarray:
    a = np.zeros(MLP_NPARAM, dtype=np.float32)
    self._raise(lib().lp_mlp_get(self._h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))
    return a


def _ctx_mlp_forward(self, feat, stream=None):
    """(z, y) of the network on feat (device, n x 16 float32)."""
    import torch
    n = feat.shape[0]
    z = torch.empty(n, dtype=torch.float32, device=feat.device)
    y = torch.empty(n, dtype=torch.float32, device=feat.device)
    self._raise(lib().lp_mlp_forward(self._h, _stream_ptr(stream), n, _ptr(feat), _ptr(z), _ptr(y)))
    return z, y


def _ctx_mlp_grad(self, feat, target, stream=None):
    """(loss, gradient) of the mean cross-entropy (host values)."""
    g = np.zeros(MLP_NPARAM, dtype=np.float32)
    loss = C.c_float(0.0)
    self._raise(lib().lp_mlp_grad(self._h, _stream_ptr(stream), feat.shape[0], _ptr(feat), _ptr(target),
                                  g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss)))
    return loss.value, g


def _ctx_mlp_train(self, feat, target, stream=None, **kw):
    """Train on (feat, target) (device tensors); returns the per-epoch mean loss."""
    t = train_cfg(**kw)
    loss = np.zeros(max(t.epochs, 1), dtype=np.float32)
    self._raise(lib().lp_mlp_train(self._h, _stream_ptr(stream), feat.shape[0], _ptr(feat), _ptr(target),
                                   C.byref(t), loss.ctypes.data_as(C.POINTER(C.c_float))))
    return loss[:t.epochs]


Context.features = _ctx_features
Context.mlp_init = _ctx_mlp_init
Context.mlp_set = _ctx_mlp_set
Context.mlp_get = _ctx_mlp_get
Context.mlp_forward = _ctx_mlp_forward
Context.mlp_grad = _ctx_mlp_grad
Context.mlp_train = _ctx_mlp_train
