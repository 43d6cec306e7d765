"""Thin ctypes binding of libqgbe (declared in include/qgbe.h).

Functions carry the C names and only marshal arguments: numpy arrays are passed
as host pointers (on_device = 0), torch tensors on the GPU as device pointers
(on_device = 1).  Every step of the computation runs in the HIP library; if the
library is missing this module raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libqgbe.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENUMERIC, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FP64, FP32 = 0, 1
SAMPLER_UNIFORM, SAMPLER_LEARNED, SAMPLER_ROOTS, SAMPLER_ROOTS_ALT = 0, 1, 2, 3
DRIFT_UPWIND, DRIFT_CENTRAL = 0, 1
MASS_DYNAMIC, MASS_CONSTANT = 0, 1
FLAG_NEGATIVE_F, FLAG_PAULI, FLAG_NONFINITE = 1, 2, 4

# every symbol include/qgbe.h declares
EXPORTS = (
    "qgbe_init_grid", "qgbe_destroy", "qgbe_last_error", "qgbe_workspace_bytes",
    "qgbe_set_distribution", "qgbe_get_distribution", "qgbe_get_masses",
    "qgbe_set_step_index", "qgbe_get_step_index", "qgbe_collision_term",
    "qgbe_collision_term_ex", "qgbe_step", "qgbe_observables", "qgbe_set_proposal_table",
    "qgbe_channel_table", "qgbe_philox4x32_10", "qgbe_proposal_set_weights",
    "qgbe_proposal_get_weights", "qgbe_mlp_forward", "qgbe_mlp_loss_grad", "qgbe_proposal_features",
    "qgbe_record_samples", "qgbe_train_proposal", "qgbe_proposal_build_table", "qgbe_get_proposal_table",
    "qgbe_checkpoint", "qgbe_restore", "qgbe_set_channel_samplers", "qgbe_get_channel_samplers",
    "qgbe_proposal_judge", "qgbe_set_matrix_element", "qgbe_collision_term_noalloc",
    "qgbe_noalloc_scratch_bytes",
)
MLP_PARAMS = 29016
MLP_BATCH = 16384
RECORD_WIDTH = 14


class QgbeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"qgbe status {status}: {msg}")
        self.status = status


class GridDesc(C.Structure):
    _fields_ = [("n_x", C.c_int32 * 3), ("n_p", C.c_int32 * 3),
                ("x_half", C.c_double * 3), ("p_half", C.c_double * 3),
                ("species_mask", C.c_uint32), ("row_mask", C.c_uint32),
                ("alpha_s", C.c_double), ("precision", C.c_int32), ("symmetric", C.c_int32),
                ("drift", C.c_int32), ("mass_mode", C.c_int32), ("const_mass2", C.c_double * 7),
                ("seed", C.c_uint64), ("device", C.c_int32), ("stream", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("N_total", C.c_double), ("N", C.c_double * 7), ("E_total", C.c_double),
                ("E", C.c_double * 7), ("P", C.c_double * 3), ("mass2_avg", C.c_double * 7),
                ("min_f", C.c_double), ("max_fermion_f", C.c_double), ("n_evals", C.c_double),
                ("t_collide_ms", C.c_double), ("t_step_ms", C.c_double), ("flags", C.c_uint32),
                ("step", C.c_uint32), ("n_accepted", C.c_double), ("mc_err_est", C.c_double),
                ("E_source", C.c_double), ("E_collide", C.c_double), ("E_total_mod", C.c_double),
                ("entropy", C.c_double), ("T_ii", C.c_double * 3),
                ("n_collide_launches", C.c_uint32), ("reserved", C.c_uint32)]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


class TrainCfg(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("lr_final", C.c_float),
                ("alpha", C.c_float), ("seed", C.c_uint64)]


class CollideExtras(C.Structure):
    _fields_ = [("scale", C.c_void_p), ("item_sums", C.c_void_p), ("on_device", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    """Load libqgbe.so (built in-tree by paper_1912_04457_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libqgbe.so not built ({LIB_PATH}); run __graft_entry__.build()")
        # PyTorch ships its own HIP runtime with the same sonames; loading it
        # first lets libqgbe bind to that one runtime instead of a second copy
        # (two runtimes in one process leave the later one without devices).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        i32, u32, p, d = C.c_int32, C.c_uint32, C.c_void_p, C.c_double
        sig = {
            "qgbe_init_grid": (i32, [p, p]),
            "qgbe_destroy": (None, [p]),
            "qgbe_last_error": (C.c_char_p, []),
            "qgbe_workspace_bytes": (C.c_size_t, [p]),
            "qgbe_set_distribution": (i32, [p, i32, p, i32]),
            "qgbe_get_distribution": (i32, [p, i32, p, i32]),
            "qgbe_get_masses": (i32, [p, p]),
            "qgbe_set_step_index": (i32, [p, u32]),
            "qgbe_get_step_index": (i32, [p, p]),
            "qgbe_collision_term": (i32, [p, i32, i32, p, i32, p]),
            "qgbe_collision_term_ex": (i32, [p, i32, i32, p, i32, p, p]),
            "qgbe_step": (i32, [p, d, i32, i32, i32, p]),
            "qgbe_observables": (i32, [p, p]),
            "qgbe_set_proposal_table": (i32, [p, i32, p, p, p, i32]),
            "qgbe_channel_table": (i32, [u32, u32, p, p, i32]),
            "qgbe_philox4x32_10": (None, [p, p, p]),
            "qgbe_proposal_set_weights": (i32, [p, p, C.c_int64]),
            "qgbe_proposal_get_weights": (i32, [p, p, C.c_int64]),
            "qgbe_mlp_forward": (i32, [p, p, C.c_int64, p, i32]),
            "qgbe_mlp_loss_grad": (i32, [p, p, p, C.c_int64, p, p, i32]),
            "qgbe_proposal_features": (i32, [p, p, i32]),
            "qgbe_record_samples": (i32, [p, i32, C.c_int64, p, C.c_int64, p, i32]),
            "qgbe_train_proposal": (i32, [p, p, C.c_int64, p, p, i32]),
            "qgbe_proposal_build_table": (i32, [p, C.c_float]),
            "qgbe_get_proposal_table": (i32, [p, p, p, p, p]),
            "qgbe_checkpoint": (i32, [p, p, p]),
            "qgbe_restore": (i32, [p, p, C.c_size_t]),
            "qgbe_set_channel_samplers": (i32, [p, p]),
            "qgbe_get_channel_samplers": (i32, [p, p]),
            "qgbe_proposal_judge": (i32, [p, i32, i32, p, p]),
            "qgbe_set_matrix_element": (i32, [p, i32, i32, p, p]),
            "qgbe_collision_term_noalloc": (i32, [p, p, u32, i32, i32, p]),
            "qgbe_noalloc_scratch_bytes": (C.c_size_t, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != OK:
        raise QgbeError(status, lib().qgbe_last_error().decode())


def _arg(x, dtype=None):
    """(pointer, on_device) of a numpy array or a torch tensor."""
    if x is None:
        return None, 0
    if isinstance(x, np.ndarray):
        if dtype is not None and x.dtype != dtype:
            raise TypeError(f"expected {dtype}, got {x.dtype}")
        if not x.flags.c_contiguous:
            raise ValueError("array must be C-contiguous")
        return x.ctypes.data_as(C.c_void_p), 0
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return C.c_void_p(x.data_ptr()), int(x.is_cuda)
    raise TypeError(f"unsupported buffer type {type(x)}")


def make_desc(*, n_x=(1, 1, 1), n_p=(10, 10, 10), x_half=(3.0, 3.0, 3.0), p_half=(2.0, 2.0, 2.0),
              species_mask=1 << 6, row_mask=0x7F, alpha_s=0.3, precision=FP64, symmetric=1,
              drift=DRIFT_UPWIND, mass_mode=MASS_DYNAMIC, const_mass2=(0.0,) * 7, seed=0x5EED2019,
              device=0, stream=None) -> GridDesc:
    d = GridDesc()
    d.n_x[:] = list(n_x)
    d.n_p[:] = list(n_p)
    d.x_half[:] = [float(v) for v in x_half]
    d.p_half[:] = [float(v) for v in p_half]
    d.species_mask = species_mask
    d.row_mask = row_mask
    d.alpha_s = alpha_s
    d.precision = precision
    d.symmetric = symmetric
    d.drift = drift
    d.mass_mode = mass_mode
    d.const_mass2[:] = [float(v) for v in const_mass2]
    d.seed = seed
    d.device = device
    d.stream = stream
    return d


# ---- functions with the C names ---------------------------------------------

def qgbe_init_grid(desc: GridDesc) -> C.c_void_p:
    ctx = C.c_void_p()
    _check(lib().qgbe_init_grid(C.byref(desc), C.byref(ctx)))
    return ctx


def qgbe_destroy(ctx) -> None:
    lib().qgbe_destroy(ctx)


def qgbe_last_error() -> str:
    return lib().qgbe_last_error().decode()


def qgbe_workspace_bytes(ctx) -> int:
    return int(lib().qgbe_workspace_bytes(ctx))


def qgbe_set_distribution(ctx, species: int, f) -> None:
    ptr, dev = _arg(f, np.float64)
    _check(lib().qgbe_set_distribution(ctx, species, ptr, dev))


def qgbe_get_distribution(ctx, species: int, f) -> None:
    ptr, dev = _arg(f, np.float64)
    _check(lib().qgbe_get_distribution(ctx, species, ptr, dev))


def qgbe_get_masses(ctx, mass2: np.ndarray) -> None:
    ptr, _ = _arg(mass2, np.float64)
    _check(lib().qgbe_get_masses(ctx, ptr))


def qgbe_set_step_index(ctx, step: int) -> None:
    _check(lib().qgbe_set_step_index(ctx, step))


def qgbe_get_step_index(ctx) -> int:
    v = C.c_uint32()
    _check(lib().qgbe_get_step_index(ctx, C.byref(v)))
    return v.value


def qgbe_collision_term(ctx, n_samples: int, sampler: int, A_out, stats: Stats | None = None) -> None:
    ptr, dev = _arg(A_out, np.float64)
    _check(lib().qgbe_collision_term(ctx, n_samples, sampler, ptr, dev,
                                     None if stats is None else C.byref(stats)))


def qgbe_collision_term_ex(ctx, n_samples: int, sampler: int, A_out, scale=None, item_sums=None,
                           stats: Stats | None = None) -> None:
    ptr, dev = _arg(A_out, np.float64)
    sp, sdev = _arg(scale, np.float64)
    ip, idev = _arg(item_sums, np.float64)
    if scale is not None and item_sums is not None and sdev != idev:
        raise ValueError("scale and item_sums must both be host or both device buffers")
    ex = CollideExtras(sp, ip, sdev if scale is not None else idev)
    _check(lib().qgbe_collision_term_ex(ctx, n_samples, sampler, ptr, dev, C.byref(ex),
                                        None if stats is None else C.byref(stats)))


def qgbe_collision_term_noalloc(desc: GridDesc, f, step: int, n_samples: int, sampler: int, A) -> None:
    """f and A: device buffers (torch tensors on desc.device)."""
    fp, fdev = _arg(f, np.float64)
    ap, adev = _arg(A, np.float64)
    if not (fdev and adev):
        raise ValueError("f and A must be device buffers")
    _check(lib().qgbe_collision_term_noalloc(C.byref(desc), fp, step, n_samples, sampler, ap))


def qgbe_noalloc_scratch_bytes() -> int:
    return int(lib().qgbe_noalloc_scratch_bytes())


def qgbe_step(ctx, dt_fm: float, n_samples: int, sampler: int, n_steps: int, per_step=None) -> None:
    _check(lib().qgbe_step(ctx, dt_fm, n_samples, sampler, n_steps, per_step))


def qgbe_observables(ctx, stats: Stats) -> None:
    _check(lib().qgbe_observables(ctx, C.byref(stats)))


def qgbe_set_proposal_table(ctx, thr, mu, sigma) -> None:
    tp, d1 = _arg(thr, np.uint32)
    mp, d2 = _arg(mu, np.float32)
    sp, d3 = _arg(sigma, np.float32)
    if not d1 == d2 == d3:
        raise ValueError("table arrays must all be host or all device buffers")
    K = int(thr.shape[-1])
    _check(lib().qgbe_set_proposal_table(ctx, K, tp, mp, sp, d1))


def qgbe_proposal_set_weights(ctx, w: np.ndarray) -> None:
    w = np.ascontiguousarray(w, dtype=np.float32)
    _check(lib().qgbe_proposal_set_weights(ctx, w.ctypes.data_as(C.c_void_p), w.size))


def qgbe_proposal_get_weights(ctx) -> np.ndarray:
    w = np.zeros(MLP_PARAMS, dtype=np.float32)
    _check(lib().qgbe_proposal_get_weights(ctx, w.ctypes.data_as(C.c_void_p), w.size))
    return w


def qgbe_mlp_forward(ctx, X, Y) -> None:
    xp, d1 = _arg(X, np.float32)
    yp, d2 = _arg(Y, np.float32)
    if d1 != d2:
        raise ValueError("X and Y must both be host or both device buffers")
    rows = X.shape[0]
    _check(lib().qgbe_mlp_forward(ctx, xp, rows, yp, d1))


def qgbe_mlp_loss_grad(ctx, X, yw, grad) -> float:
    xp, d1 = _arg(X, np.float32)
    wp, d2 = _arg(yw, np.float32)
    gp, d3 = _arg(grad, np.float32)
    if not d1 == d2 == d3:
        raise ValueError("buffers must all be host or all device")
    loss = C.c_double()
    _check(lib().qgbe_mlp_loss_grad(ctx, xp, wp, X.shape[0], gp, C.byref(loss), d1))
    return loss.value


def qgbe_proposal_features(ctx, X) -> None:
    xp, dev = _arg(X, np.float32)
    _check(lib().qgbe_proposal_features(ctx, xp, dev))


def qgbe_record_samples(ctx, n_per_item: int, item_stride: int, rows) -> int:
    rp, dev = _arg(rows, np.float32)
    n = C.c_int64()
    max_rows = (rows.numel() if hasattr(rows, "numel") else rows.size) // RECORD_WIDTH
    _check(lib().qgbe_record_samples(ctx, n_per_item, item_stride, rp, max_rows, C.byref(n), dev))
    return n.value


def qgbe_train_proposal(ctx, rows, cfg: TrainCfg, epoch_loss: np.ndarray | None = None) -> None:
    rp, dev = _arg(rows, np.float32)
    n = (rows.numel() if hasattr(rows, "numel") else rows.size) // RECORD_WIDTH
    lp = None if epoch_loss is None else epoch_loss.ctypes.data_as(C.c_void_p)
    _check(lib().qgbe_train_proposal(ctx, rp, n, C.byref(cfg), lp, dev))


def qgbe_proposal_build_table(ctx, alpha: float = 0.1) -> None:
    _check(lib().qgbe_proposal_build_table(ctx, alpha))


def qgbe_get_proposal_table(ctx, rows: int):
    K = C.c_int32()
    _check(lib().qgbe_get_proposal_table(ctx, C.byref(K), None, None, None))
    thr = np.zeros((rows, K.value), dtype=np.uint32)
    mu = np.zeros((rows, K.value, 5), dtype=np.float32)
    sg = np.zeros((rows, K.value, 5), dtype=np.float32)
    _check(lib().qgbe_get_proposal_table(ctx, C.byref(K), thr.ctypes.data_as(C.c_void_p),
                                         mu.ctypes.data_as(C.c_void_p), sg.ctypes.data_as(C.c_void_p)))
    return thr, mu, sg


def qgbe_checkpoint(ctx) -> bytes:
    """The context's state as a byte string (see qgbe_restore)."""
    n = C.c_size_t(0)
    _check(lib().qgbe_checkpoint(ctx, None, C.byref(n)))
    buf = C.create_string_buffer(n.value)
    _check(lib().qgbe_checkpoint(ctx, buf, C.byref(n)))
    return buf.raw[:n.value]


def qgbe_restore(ctx, state: bytes) -> None:
    buf = C.create_string_buffer(state, len(state))
    _check(lib().qgbe_restore(ctx, buf, len(state)))


def qgbe_set_channel_samplers(ctx, use_learned) -> None:
    v = np.ascontiguousarray(use_learned, dtype=np.uint8)
    _check(lib().qgbe_set_channel_samplers(ctx, v.ctypes.data_as(C.c_void_p)))


def qgbe_get_channel_samplers(ctx, n_channels: int) -> np.ndarray:
    v = np.zeros(n_channels, dtype=np.uint8)
    _check(lib().qgbe_get_channel_samplers(ctx, v.ctypes.data_as(C.c_void_p)))
    return v


def qgbe_set_matrix_element(ctx, row: int, terms) -> None:
    """terms = [(coef, (a, b, c, d, e, f)), ...] (see include/qgbe.h); [] restores Table I."""
    coef = np.ascontiguousarray([t[0] for t in terms], dtype=np.float64)
    powers = np.ascontiguousarray([t[1] for t in terms], dtype=np.int32).reshape(-1, 6)
    _check(lib().qgbe_set_matrix_element(ctx, row, len(terms), coef.ctypes.data_as(C.c_void_p),
                                         powers.ctypes.data_as(C.c_void_p)))


def qgbe_proposal_judge(ctx, n_pilot: int, n_reps: int, n_channels: int):
    """Run the fallback judge; returns (use_learned [channels] uint8, ratio [channels])."""
    flags = np.zeros(n_channels, dtype=np.uint8)
    ratio = np.zeros(n_channels)
    _check(lib().qgbe_proposal_judge(ctx, n_pilot, n_reps, flags.ctypes.data_as(C.c_void_p),
                                     ratio.ctypes.data_as(C.c_void_p)))
    return flags, ratio


def qgbe_channel_table(species_mask: int, row_mask: int = 0x7F):
    rows = np.zeros((70, 5), dtype=np.int32)
    w = np.zeros((70, 2), dtype=np.float64)
    n = lib().qgbe_channel_table(species_mask, row_mask, rows.ctypes.data_as(C.c_void_p),
                                 w.ctypes.data_as(C.c_void_p), 70)
    if n < 0:
        raise QgbeError(n, qgbe_last_error())
    return rows[:n], w[:n]


def qgbe_philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().qgbe_philox4x32_10(c.ctypes.data_as(C.c_void_p), k.ctypes.data_as(C.c_void_p),
                             out.ctypes.data_as(C.c_void_p))
    return out


class Solver:
    """Owns one context; convenience methods over the C calls."""

    def __init__(self, **desc_kw):
        self.desc = make_desc(**desc_kw)
        self.ctx = qgbe_init_grid(self.desc)
        self.cells = int(np.prod(desc_kw.get("n_x", (1, 1, 1))))
        self.nodes = int(np.prod(desc_kw.get("n_p", (10, 10, 10))))
        self.n_channels = len(qgbe_channel_table(self.desc.species_mask, self.desc.row_mask)[0])

    def close(self):
        if self.ctx:
            qgbe_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _expect(self, x, species: int):
        want = (7 if species < 0 else 1) * self.cells * self.nodes
        n = x.numel() if hasattr(x, "numel") else x.size
        if n != want:
            raise ValueError(f"expected {want} values for species {species}, got {n}")

    def set_f(self, f, species: int = -1):
        self._expect(f, species)
        qgbe_set_distribution(self.ctx, species, f)

    def get_f(self) -> np.ndarray:
        out = np.zeros((7, self.cells, self.nodes))
        qgbe_get_distribution(self.ctx, -1, out)
        return out

    def masses(self) -> np.ndarray:
        out = np.zeros((7, self.cells))
        qgbe_get_masses(self.ctx, out)
        return out

    def collision(self, n_samples: int, *, sampler: int = SAMPLER_UNIFORM, scale: bool = False,
                  items: bool = False):
        A = np.zeros((7, self.cells, self.nodes))
        S = np.zeros_like(A) if scale else None
        I = np.zeros((self.cells, self.n_channels, self.nodes)) if items else None
        st = Stats()
        qgbe_collision_term_ex(self.ctx, n_samples, sampler, A, S, I, st)
        return A, S, I, st

    def observables(self) -> dict:
        st = Stats()
        qgbe_observables(self.ctx, st)
        return st.as_dict()

    def step(self, dt_fm: float, n_samples: int, n_steps: int = 1, sampler: int = SAMPLER_UNIFORM,
             last_only: bool = False):
        """n_steps steps; the statistics of every step, or with last_only those
        of the last one only (the steps before run without the per-step
        reductions and host synchronisation)."""
        if last_only and n_steps > 1:
            qgbe_step(self.ctx, dt_fm, n_samples, sampler, n_steps - 1, None)
            n_steps = 1
        stats = (Stats * n_steps)()
        qgbe_step(self.ctx, dt_fm, n_samples, sampler, n_steps, stats)
        return [s.as_dict() for s in stats]
