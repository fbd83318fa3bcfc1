"""Python binding of libtla: batched small dense solvers on MI355X.

Thin ctypes layer over the C ABI in include/tla.h (same entry-point names);
it only marshals arguments.  Every step of the solvers runs in the HIP
kernels of libtla.so; PyTorch supplies device memory and streams.  There is
no CPU fallback: if the library is not built, loading it raises.

Matrix convention on the device ("column-major batch"): a float64 CUDA tensor
M of shape (batch, n, ld) holds instance b's element (i, j) at M[b, j, i],
i.e. each instance is stored column-major with leading dimension ld.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libtla.so")

# enums of tla.h
F64, MIXED_F32, MIXED_F16, MIXED_BF16 = 0, 1, 2, 3
POTRF, TRSYL, TRLYAP = 0, 1, 2
PICK_DEFAULT, PICK_TABLE, PICK_MLP = 0, 1, 2
STAT_CONVERGED, STAT_FALLBACK, STAT_BREAKDOWN, STAT_NONFINITE = 1, 2, 4, 8
OK, E_ARG, E_HIP, E_NOMEM, E_UNSUPPORTED = 0, 1, 2, 3, 4
PRECS = {"f64": F64, "mixed_f32": MIXED_F32, "mixed_f16": MIXED_F16, "mixed_bf16": MIXED_BF16}
OPS = {"potrf": POTRF, "trsyl": TRSYL, "trlyap": TRLYAP}

# every exported symbol of include/tla.h
SYMBOLS = [
    "tla_create", "tla_destroy", "tla_set_stream", "tla_sync",
    "tla_potrf_batched", "tla_trsyl_batched", "tla_trlyap_batched", "tla_ragged_batched", "tla_ragged_batched_noalloc",
    "tla_potrs_batched", "tla_potri_batched", "tla_gesyl_batched", "tla_gelyap_batched",
    "tla_spotrf_batched", "tla_strsyl_batched", "tla_strlyap_batched", "tla_set_plan", "tla_get_plan", "tla_num_candidates", "tla_candidate", "tla_variant_name",
    "tla_tune", "tla_time_plan", "tla_save_table", "tla_load_table", "tla_set_picker",
    "tla_set_refine", "tla_status_string",
    "tla_mlp_num_params", "tla_mlp_num_features", "tla_mlp_features", "tla_mlp_set_params",
    "tla_mlp_get_params", "tla_mlp_forward_backward", "tla_mlp_adam_step", "tla_mlp_train",
    "tla_mlp_predict", "tla_mlp_save", "tla_mlp_load", "tla_set_picker_judge", "tla_picker_judge_stats",
    "tla_set_exact_size", "tla_exact_size_stats",
]


class TlaError(RuntimeError):
    pass


class Plan(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int), ("tile", ctypes.c_int), ("engine", ctypes.c_int),
                ("waves", ctypes.c_int), ("place", ctypes.c_int)]

    def __repr__(self):
        return (f"Plan(variant={self.variant}, tile={self.tile}, engine={self.engine}, waves={self.waves}, "
                f"place={self.place})")

    def astuple(self):
        return (self.variant, self.tile, self.engine, self.waves, self.place)


class Desc(ctypes.Structure):
    """tla_desc: one ragged work item."""
    _fields_ = [("op", ctypes.c_int), ("n", ctypes.c_int), ("lda", ctypes.c_int), ("ldb", ctypes.c_int),
                ("ldc", ctypes.c_int), ("pad_", ctypes.c_int), ("a", ctypes.c_uint64),
                ("b", ctypes.c_uint64), ("c", ctypes.c_uint64)]


DESC_NP = np.dtype([("op", np.int32), ("n", np.int32), ("lda", np.int32), ("ldb", np.int32),
                    ("ldc", np.int32), ("pad_", np.int32), ("a", np.uint64), ("b", np.uint64),
                    ("c", np.uint64)])
STAT_NP = np.dtype([("iters", np.int32), ("flags", np.int32), ("eta", np.float64)])

_lib = None


def lib():
    """Load libtla.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise TlaError(f"libtla.so not built at {LIB_PATH}; run python -m paper_1906_08613_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, I, V = ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p
        D = ctypes.c_double
        sig = {
            "tla_create": (I, [ctypes.POINTER(V), I]),
            "tla_destroy": (I, [V]),
            "tla_set_stream": (I, [V, V]),
            "tla_sync": (I, [V]),
            "tla_potrf_batched": (I, [V, I, I, I, P, P, P, P, P]),
            "tla_trsyl_batched": (I, [V, I, I, I, P, P, P, P, P, P, P, P, P]),
            "tla_trlyap_batched": (I, [V, I, I, I, P, P, P, P, P, P, P]),
            "tla_gesyl_batched": (I, [V, I, I, I, P, P, P, P, P, P, P, P, P]),
            "tla_gelyap_batched": (I, [V, I, I, I, P, P, P, P, P, P, P]),
            "tla_ragged_batched": (I, [V, I, I, I, P, P, P]),
            "tla_ragged_batched_noalloc": (I, [V, I, I, I, P, P, P]),
            "tla_potrs_batched": (I, [V, I, I, P, I, P, P, P, P, P, P]),
            "tla_potri_batched": (I, [V, I, I, P, P, P, P, P, P]),
            "tla_spotrf_batched": (I, [V, I, I, P, P, P, P]),
            "tla_strsyl_batched": (I, [V, I, I, P, P, P, P, P, P, P, P]),
            "tla_strlyap_batched": (I, [V, I, I, P, P, P, P, P, P]),
            "tla_set_plan": (I, [V, I, I, ctypes.POINTER(Plan)]),
            "tla_get_plan": (I, [V, I, I, I, I, ctypes.POINTER(Plan)]),
            "tla_num_candidates": (I, [I]),
            "tla_candidate": (I, [I, I, ctypes.POINTER(Plan)]),
            "tla_variant_name": (ctypes.c_char_p, [I, I]),
            "tla_tune": (I, [V, I, P, I, P, I, P, I, I]),
            "tla_time_plan": (I, [V, I, I, I, I, ctypes.POINTER(Plan), I, ctypes.POINTER(D)]),
            "tla_save_table": (I, [V, ctypes.c_char_p]),
            "tla_load_table": (I, [V, ctypes.c_char_p]),
            "tla_set_picker": (I, [V, I]),
            "tla_set_refine": (I, [V, D, I]),
            "tla_status_string": (ctypes.c_char_p, [I]),
            "tla_mlp_num_params": (I, []),
            "tla_mlp_num_features": (I, []),
            "tla_mlp_features": (I, [I, I, I, I, ctypes.POINTER(Plan), P]),
            "tla_mlp_set_params": (I, [V, P]),
            "tla_mlp_get_params": (I, [V, P]),
            "tla_mlp_forward_backward": (I, [V, I, P, P, P, P, P]),
            "tla_mlp_adam_step": (I, [V, P, ctypes.c_float]),
            "tla_mlp_train": (I, [V, I, ctypes.c_float, ctypes.c_ulonglong, I, P]),
            "tla_mlp_predict": (I, [V, I, I, I, I, ctypes.POINTER(Plan), ctypes.POINTER(D)]),
            "tla_mlp_save": (I, [V, ctypes.c_char_p]),
            "tla_set_picker_judge": (I, [V, D, I]),
            "tla_set_exact_size": (I, [V, I]),
            "tla_exact_size_stats": (I, [V, ctypes.POINTER(I), ctypes.POINTER(I)]),
            "tla_picker_judge_stats": (I, [V, ctypes.POINTER(I), ctypes.POINTER(I)]),
            "tla_mlp_load": (I, [V, ctypes.c_char_p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int, what: str = "tla call"):
    if status != OK:
        msg = lib().tla_status_string(status).decode()
        raise TlaError(f"{what}: {msg} ({status})")


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _prec(p):
    return PRECS[p] if isinstance(p, str) else int(p)


# ------------------------------------------------------------------ handle
class Handle:
    """Owns a tla_handle bound to a device; work goes on torch's current stream
    unless `stream` is given."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.device = device
        h = ctypes.c_void_p()
        check(lib().tla_create(ctypes.byref(h), device), "tla_create")
        self.h = h
        self.set_stream(stream if stream is not None else torch.cuda.current_stream(device))

    def set_stream(self, stream):
        self.stream = stream
        check(lib().tla_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)), "tla_set_stream")

    def close(self):
        if getattr(self, "h", None):
            lib().tla_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        check(lib().tla_sync(self.h), "tla_sync")

    # --------------------------------------------------- raw C-ABI calls
    def potrf_batched(self, prec, batch, n_max, n, A, lda, info, stat=None):
        check(lib().tla_potrf_batched(self.h, _prec(prec), batch, n_max, _ptr(n), _ptr(A), _ptr(lda),
                                      _ptr(info), _ptr(stat)), "tla_potrf_batched")

    def trsyl_batched(self, prec, batch, n_max, n, L, ldl, U, ldu, C, ldc, info, stat=None):
        check(lib().tla_trsyl_batched(self.h, _prec(prec), batch, n_max, _ptr(n), _ptr(L), _ptr(ldl),
                                      _ptr(U), _ptr(ldu), _ptr(C), _ptr(ldc), _ptr(info), _ptr(stat)),
              "tla_trsyl_batched")

    def gesyl_batched(self, prec, batch, n_max, n, A, lda, B, ldb, C, ldc, info, stat=None):
        check(lib().tla_gesyl_batched(self.h, _prec(prec), batch, n_max, _ptr(n), _ptr(A), _ptr(lda),
                                      _ptr(B), _ptr(ldb), _ptr(C), _ptr(ldc), _ptr(info), _ptr(stat)),
              "tla_gesyl_batched")

    def gelyap_batched(self, prec, batch, n_max, n, A, lda, S, lds, info, stat=None):
        check(lib().tla_gelyap_batched(self.h, _prec(prec), batch, n_max, _ptr(n), _ptr(A), _ptr(lda),
                                       _ptr(S), _ptr(lds), _ptr(info), _ptr(stat)), "tla_gelyap_batched")

    def trlyap_batched(self, prec, batch, n_max, n, L, ldl, S, lds, info, stat=None):
        check(lib().tla_trlyap_batched(self.h, _prec(prec), batch, n_max, _ptr(n), _ptr(L), _ptr(ldl),
                                       _ptr(S), _ptr(lds), _ptr(info), _ptr(stat)), "tla_trlyap_batched")

    def potrs_batched(self, batch, n_max, n, nrhs_max, nrhs, X, ldx, B, ldb, info):
        check(lib().tla_potrs_batched(self.h, batch, n_max, _ptr(n), nrhs_max, _ptr(nrhs), _ptr(X), _ptr(ldx),
                                      _ptr(B), _ptr(ldb), _ptr(info)), "tla_potrs_batched")

    def potri_batched(self, batch, n_max, n, X, ldx, Y, ldy, info):
        check(lib().tla_potri_batched(self.h, batch, n_max, _ptr(n), _ptr(X), _ptr(ldx), _ptr(Y), _ptr(ldy),
                                      _ptr(info)), "tla_potri_batched")

    def spotrf_batched(self, batch, n_max, n, A, lda, info):
        check(lib().tla_spotrf_batched(self.h, batch, n_max, _ptr(n), _ptr(A), _ptr(lda), _ptr(info)),
              "tla_spotrf_batched")

    def strsyl_batched(self, batch, n_max, n, L, ldl, U, ldu, C, ldc, info):
        check(lib().tla_strsyl_batched(self.h, batch, n_max, _ptr(n), _ptr(L), _ptr(ldl), _ptr(U), _ptr(ldu),
                                       _ptr(C), _ptr(ldc), _ptr(info)), "tla_strsyl_batched")

    def strlyap_batched(self, batch, n_max, n, L, ldl, S, lds, info):
        check(lib().tla_strlyap_batched(self.h, batch, n_max, _ptr(n), _ptr(L), _ptr(ldl), _ptr(S), _ptr(lds),
                                        _ptr(info)), "tla_strlyap_batched")

    def ragged_batched(self, prec, batch, n_max, desc, info, stat=None):
        check(lib().tla_ragged_batched(self.h, _prec(prec), batch, n_max, _ptr(desc), _ptr(info), _ptr(stat)),
              "tla_ragged_batched")

    def ragged_batched_noalloc(self, prec, batch, n_max, desc, info, stat=None):
        check(lib().tla_ragged_batched_noalloc(self.h, _prec(prec), batch, n_max, _ptr(desc), _ptr(info),
                                               _ptr(stat)), "tla_ragged_batched_noalloc")

    # ------------------------------------------------------------- plans
    def set_plan(self, op, prec, plan=None):
        if plan is None:
            p = Plan(-1, 16, 1, 4, 0)
        else:
            p = Plan(*plan) if not isinstance(plan, Plan) else plan
        check(lib().tla_set_plan(self.h, OPS.get(op, op), _prec(prec), ctypes.byref(p)), "tla_set_plan")

    def get_plan(self, op, n, prec, batch):
        p = Plan()
        check(lib().tla_get_plan(self.h, OPS.get(op, op), n, _prec(prec), batch, ctypes.byref(p)), "tla_get_plan")
        return p

    def set_picker(self, mode):
        check(lib().tla_set_picker(self.h, mode), "tla_set_picker")

    def set_refine(self, tau=1e-13, max_iter=8):
        check(lib().tla_set_refine(self.h, tau, max_iter), "tla_set_refine")

    def time_plan(self, op, n, prec, batch, plan, reps=5):
        p = Plan(*plan) if not isinstance(plan, Plan) else plan
        s = ctypes.c_double()
        check(lib().tla_time_plan(self.h, OPS.get(op, op), n, _prec(prec), batch, ctypes.byref(p), reps,
                                  ctypes.byref(s)), "tla_time_plan")
        return s.value

    def tune(self, ops, ns, precs, batch=1024, reps=3):
        a = np.array([OPS.get(o, o) for o in ops], dtype=np.int32)
        b = np.array(ns, dtype=np.int32)
        c = np.array([_prec(p) for p in precs], dtype=np.int32)
        check(lib().tla_tune(self.h, len(a), a.ctypes.data_as(ctypes.c_void_p), len(b),
                             b.ctypes.data_as(ctypes.c_void_p), len(c), c.ctypes.data_as(ctypes.c_void_p),
                             batch, reps), "tla_tune")

    # ------------------------------------------------- learned cost model
    def mlp_set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        check(lib().tla_mlp_set_params(self.h, p.ctypes.data_as(ctypes.c_void_p)), "tla_mlp_set_params")

    def mlp_get_params(self):
        p = np.zeros(mlp_num_params(), dtype=np.float32)
        check(lib().tla_mlp_get_params(self.h, p.ctypes.data_as(ctypes.c_void_p)), "tla_mlp_get_params")
        return p

    def mlp_forward_backward(self, X, T):
        X = np.ascontiguousarray(X, dtype=np.float32)
        T = np.ascontiguousarray(T, dtype=np.float32)
        N = X.shape[0]
        loss = np.zeros(1, dtype=np.float32)
        grad = np.zeros(mlp_num_params(), dtype=np.float32)
        Y = np.zeros(N, dtype=np.float32)
        vp = ctypes.c_void_p
        check(lib().tla_mlp_forward_backward(self.h, N, X.ctypes.data_as(vp), T.ctypes.data_as(vp),
                                             loss.ctypes.data_as(vp), grad.ctypes.data_as(vp),
                                             Y.ctypes.data_as(vp)), "tla_mlp_forward_backward")
        return float(loss[0]), grad, Y

    def mlp_adam_step(self, grad, lr):
        g = np.ascontiguousarray(grad, dtype=np.float32)
        check(lib().tla_mlp_adam_step(self.h, g.ctypes.data_as(ctypes.c_void_p), lr), "tla_mlp_adam_step")

    def mlp_train(self, epochs=2000, lr=3e-3, seed=1, exclude_mod=0):
        loss = np.zeros(1, dtype=np.float32)
        check(lib().tla_mlp_train(self.h, epochs, lr, seed, exclude_mod, loss.ctypes.data_as(ctypes.c_void_p)),
              "tla_mlp_train")
        return float(loss[0])

    def mlp_predict(self, op, n, prec, batch, plan):
        p = Plan(*plan) if not isinstance(plan, Plan) else plan
        s = ctypes.c_double()
        check(lib().tla_mlp_predict(self.h, OPS.get(op, op), n, _prec(prec), batch, ctypes.byref(p),
                                    ctypes.byref(s)), "tla_mlp_predict")
        return s.value

    def mlp_save(self, path):
        check(lib().tla_mlp_save(self.h, path.encode()), "tla_mlp_save")

    def mlp_load(self, path):
        check(lib().tla_mlp_load(self.h, path.encode()), "tla_mlp_load")

    def set_exact_size(self, mode):
        """0 / False: off; 1 / True: always; 2: where measured faster."""
        check(lib().tla_set_exact_size(self.h, int(mode)), "tla_set_exact_size")

    def exact_size_stats(self):
        c, f = ctypes.c_int(0), ctypes.c_int(0)
        check(lib().tla_exact_size_stats(self.h, ctypes.byref(c), ctypes.byref(f)), "tla_exact_size_stats")
        return c.value, f.value

    def set_picker_judge(self, margin, max_timed=4):
        check(lib().tla_set_picker_judge(self.h, float(margin), int(max_timed)), "tla_set_picker_judge")

    def picker_judge_stats(self):
        j, m = ctypes.c_int(0), ctypes.c_int(0)
        check(lib().tla_picker_judge_stats(self.h, ctypes.byref(j), ctypes.byref(m)), "tla_picker_judge_stats")
        return j.value, m.value

    def save_table(self, path):
        check(lib().tla_save_table(self.h, path.encode()), "tla_save_table")

    def load_table(self, path):
        check(lib().tla_load_table(self.h, path.encode()), "tla_load_table")


def num_candidates(op):
    return lib().tla_num_candidates(OPS.get(op, op))


def candidate(op, i):
    p = Plan()
    check(lib().tla_candidate(OPS.get(op, op), i, ctypes.byref(p)), "tla_candidate")
    return p


def mlp_num_params():
    return lib().tla_mlp_num_params()


def mlp_num_features():
    return lib().tla_mlp_num_features()


def mlp_features(op, n, prec, batch, plan):
    p = Plan(*plan) if not isinstance(plan, Plan) else plan
    f = np.zeros(mlp_num_features(), dtype=np.float32)
    check(lib().tla_mlp_features(OPS.get(op, op), n, _prec(prec), batch, ctypes.byref(p),
                                 f.ctypes.data_as(ctypes.c_void_p)), "tla_mlp_features")
    return f


def variant_name(op, v):
    return lib().tla_variant_name(OPS.get(op, op), v).decode()


def num_variants(op):
    """Number of variants of op (names are valid for 0..count-1): the blocked
    algorithms, then (Sylvester, Lyapunov) the splitting-iteration solve of the
    mixed precisions."""
    v = 0
    while variant_name(op, v) != "invalid":
        v += 1
    return v


def blocked_variants(op):
    """Indices of the blocked-algorithm variants of op (every precision and size)."""
    return [v for v in range(num_variants(op)) if variant_name(op, v) != "jacobi-sweeps"]


# ---------------------------------------------------------- batch helpers
def to_device_cm(M, device="cuda", ld=None, dtype=np.float64):
    """numpy (batch, n, n) indexed [b, i, j] -> column-major batch tensor (batch, n, ld)."""
    import torch
    M = np.asarray(M, dtype=dtype)
    b, n = M.shape[0], M.shape[-1]
    ld = ld or n
    host = np.zeros((b, n, ld), dtype=dtype)
    host[:, :, :n] = np.swapaxes(M, 1, 2)
    return torch.from_numpy(host).to(device)


def from_device_cm(t, n=None):
    """column-major batch tensor (batch, n, ld) -> numpy (batch, n, n) indexed [b, i, j]."""
    a = t.detach().cpu().numpy()
    n = n or a.shape[1]
    return np.ascontiguousarray(np.swapaxes(a[:, :n, :n], 1, 2))


def to_device_rect(M, device="cuda", ld=None):
    """numpy (batch, n, m) indexed [b, i, j] -> column-major batch tensor (batch, m, ld)."""
    import torch
    M = np.asarray(M, dtype=np.float64)
    b, n, m = M.shape
    ld = ld or n
    host = np.zeros((b, m, ld), dtype=np.float64)
    host[:, :, :n] = np.swapaxes(M, 1, 2)
    return torch.from_numpy(host).to(device)


def from_device_rect(t, n):
    """column-major batch tensor (batch, m, ld) -> numpy (batch, n, m) indexed [b, i, j]."""
    a = t.detach().cpu().numpy()
    return np.ascontiguousarray(np.swapaxes(a[:, :, :n], 1, 2))


class Operands:
    """Device arrays describing one uniform batch: per-instance n and ld
    (int32) and pointer arrays (int64 device addresses) for each matrix."""

    def __init__(self, n, *mats, device="cuda"):
        import torch
        self.mats = mats
        self.batch = mats[0].shape[0]
        self.n_max = n
        self.n = torch.full((self.batch,), n, dtype=torch.int32, device=device)
        self.ptrs, self.lds = [], []
        for m in mats:
            assert m.dtype in (torch.float64, torch.float32) and m.is_contiguous() and m.shape[0] == self.batch
            stride = m.shape[1] * m.shape[2] * m.element_size()
            base = m.data_ptr()
            p = torch.arange(self.batch, dtype=torch.int64, device=device) * stride + base
            self.ptrs.append(p)
            self.lds.append(torch.full((self.batch,), m.shape[2], dtype=torch.int32, device=device))
        self.info = torch.zeros(self.batch, dtype=torch.int32, device=device)
        self.stat = torch.zeros((self.batch, 2), dtype=torch.float64, device=device)  # 16 B per tla_stat


def stat_view(stat_tensor):
    """(batch, 2) float64 tensor holding tla_stat records -> structured numpy array."""
    return stat_tensor.detach().cpu().numpy().view(STAT_NP).reshape(-1)


def potrf(h: Handle, A, prec="f64", ops: Operands | None = None):
    """In place on the column-major batch A (batch, n, ld)."""
    ops = ops or Operands(A.shape[1], A)
    h.potrf_batched(prec, ops.batch, ops.n_max, ops.n, ops.ptrs[0], ops.lds[0], ops.info, ops.stat)
    return ops


def trsyl(h: Handle, L, U, C, prec="f64", ops: Operands | None = None):
    ops = ops or Operands(C.shape[1], L, U, C)
    h.trsyl_batched(prec, ops.batch, ops.n_max, ops.n, ops.ptrs[0], ops.lds[0], ops.ptrs[1], ops.lds[1],
                    ops.ptrs[2], ops.lds[2], ops.info, ops.stat)
    return ops


def trlyap(h: Handle, L, S, prec="f64", ops: Operands | None = None):
    ops = ops or Operands(S.shape[1], L, S)
    h.trlyap_batched(prec, ops.batch, ops.n_max, ops.n, ops.ptrs[0], ops.lds[0], ops.ptrs[1], ops.lds[1],
                     ops.info, ops.stat)
    return ops


def gesyl(h: Handle, A, B, C, prec="f64", ops: Operands | None = None):
    """General Sylvester A X + X B = C (real spectra), C overwritten with X."""
    ops = ops or Operands(C.shape[1], A, B, C)
    h.gesyl_batched(prec, ops.batch, ops.n_max, ops.n, ops.ptrs[0], ops.lds[0], ops.ptrs[1], ops.lds[1],
                    ops.ptrs[2], ops.lds[2], ops.info, ops.stat)
    return ops


def gelyap(h: Handle, A, S, prec="f64", ops: Operands | None = None):
    """General Lyapunov A X + X A^T = S (lower triangle of S read), S overwritten with X."""
    ops = ops or Operands(S.shape[1], A, S)
    h.gelyap_batched(prec, ops.batch, ops.n_max, ops.n, ops.ptrs[0], ops.lds[0], ops.ptrs[1], ops.lds[1],
                     ops.info, ops.stat)
    return ops


def spotrf(h: Handle, A, ops: Operands | None = None):
    """FP32 I/O and arithmetic, in place on the float32 column-major batch A (batch, n, ld)."""
    ops = ops or Operands(A.shape[1], A)
    h.spotrf_batched(ops.batch, ops.n_max, ops.n, ops.ptrs[0], ops.lds[0], ops.info)
    return ops


def strsyl(h: Handle, L, U, C, ops: Operands | None = None):
    ops = ops or Operands(C.shape[1], L, U, C)
    h.strsyl_batched(ops.batch, ops.n_max, ops.n, ops.ptrs[0], ops.lds[0], ops.ptrs[1], ops.lds[1],
                     ops.ptrs[2], ops.lds[2], ops.info)
    return ops


def strlyap(h: Handle, L, S, ops: Operands | None = None):
    ops = ops or Operands(S.shape[1], L, S)
    h.strlyap_batched(ops.batch, ops.n_max, ops.n, ops.ptrs[0], ops.lds[0], ops.ptrs[1], ops.lds[1], ops.info)
    return ops


def potrs(h: Handle, X, B, n):
    """In place on B: B := (X^T X)^{-1} B for column-major batches X (batch, n, ldx) holding
    upper factors and B (batch, m, ldb) holding n x m right-hand sides."""
    import torch
    ox = Operands(n, X)
    batch, m = B.shape[0], B.shape[1]
    ob = Operands(n, B)
    nrhs = torch.full((batch,), m, dtype=torch.int32, device=B.device)
    h.potrs_batched(batch, n, ox.n, m, nrhs, ox.ptrs[0], ox.lds[0], ob.ptrs[0], ob.lds[0], ob.info)
    return ob


def potri(h: Handle, X, Y, n):
    """Y := (X^T X)^{-1} for column-major batches X (batch, n, ldx) holding upper factors and
    Y (batch, n, ldy)."""
    ox, oy = Operands(n, X), Operands(n, Y)
    h.potri_batched(ox.batch, n, ox.n, ox.ptrs[0], ox.lds[0], oy.ptrs[0], oy.lds[0], oy.info)
    return oy


class RaggedBatch:
    """Device storage and tla_desc array for a ragged batch.

    ops: sequence of POTRF/TRSYL/TRLYAP; mats[b]: tuple of numpy matrices of
    instance b in the roles of tla_desc (potrf: (A,), trsyl: (L, U, C),
    trlyap: (L, S)), indexed [i, j].  All matrices of all instances share one
    flat float64 device buffer, each stored column-major with ld = n + pad.
    """

    def __init__(self, ops, mats, device="cuda", pad=0):
        import torch
        self.ops = [int(o) for o in ops]
        self.batch = len(self.ops)
        sizes, offs = [], []
        total = 0
        for b, m in enumerate(mats):
            n = m[0].shape[-1]
            ld = n + pad
            o = []
            for _ in m:
                o.append(total)
                total += max(ld * n, 1)
            offs.append(o)
            sizes.append((n, ld))
        host = np.zeros(max(total, 1), dtype=np.float64)
        for b, m in enumerate(mats):
            n, ld = sizes[b]
            for k, M in enumerate(m):
                blk = np.zeros((n, ld))
                blk[:, :n] = np.asarray(M, dtype=np.float64).T
                host[offs[b][k]:offs[b][k] + ld * n] = blk.reshape(-1)
        self.buf = torch.from_numpy(host).to(device)
        base = self.buf.data_ptr()
        d = np.zeros(self.batch, dtype=DESC_NP)
        for b in range(self.batch):
            n, ld = sizes[b]
            d["op"][b] = self.ops[b]
            d["n"][b] = n
            d["lda"][b] = d["ldb"][b] = d["ldc"][b] = ld
            ptr = [base + 8 * o for o in offs[b]]
            if self.ops[b] == POTRF:
                d["a"][b] = ptr[0]
            elif self.ops[b] == TRSYL:
                d["a"][b], d["b"][b], d["c"][b] = ptr
            else:
                d["a"][b], d["c"][b] = ptr
        self.sizes, self.offs = sizes, offs
        self.desc_host = d
        self.desc = torch.from_numpy(d.view(np.uint8).copy()).to(device)
        self.info = torch.zeros(self.batch, dtype=torch.int32, device=device)
        self.stat = torch.zeros((self.batch, 2), dtype=torch.float64, device=device)
        self.n_max = max([s[0] for s in sizes] + [0])

    def result(self, b):
        """Output matrix of instance b (numpy, [i, j]): A/X for potrf, X otherwise."""
        n, ld = self.sizes[b]
        k = 0 if self.ops[b] == POTRF else len(self.offs[b]) - 1
        o = self.offs[b][k]
        blk = self.buf[o:o + ld * n].view(n, ld).cpu().numpy()
        return np.ascontiguousarray(blk[:, :n].T)


def ragged(h: Handle, rb: RaggedBatch, prec="f64", n_max=None):
    h.ragged_batched(prec, rb.batch, rb.n_max if n_max is None else n_max, rb.desc, rb.info, rb.stat)
    return rb


def ragged_noalloc(h: Handle, rb: RaggedBatch, prec="f64", n_max=None):
    """The allocation-free ragged entry point (FP64, batch <= 1048576)."""
    h.ragged_batched_noalloc(prec, rb.batch, rb.n_max if n_max is None else n_max, rb.desc, rb.info, rb.stat)
    return rb
