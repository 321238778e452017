"""Python binding of libpmh.so (the C ABI in include/pmh.h).

Argument marshalling only: torch tensors supply device memory and the current
stream; every step of the signature computation runs in the HIP library.  The
binding raises if the library is missing or no GPU is present; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PMH_LIB=stats selects the event-counting build libpmh_stats.so (schedule
# analysis only; same kernels with counters)
LIB_PATH = os.path.join(_HERE, "libpmh_stats.so" if os.environ.get("PMH_LIB") == "stats" else "libpmh.so")

PMH_OK, PMH_ERR_ARG, PMH_ERR_M_RANGE, PMH_ERR_VARIANT_M, PMH_ERR_WEIGHT = 0, 1, 2, 3, 4
PMH_ERR_SET_TOO_LARGE, PMH_ERR_DEVICE, PMH_ERR_OOM, PMH_ERR_BUSY, PMH_ERR_NOT_READY = 5, 6, 7, 8, 9
PMH_ERR_SCRATCH_LIMIT, PMH_ERR_NO_ENTRY = 10, 11
IDX_EMPTY = 0xFFFFFFFF
KEY_EMPTY = 0xFFFFFFFFFFFFFFFF

_lib = None

# every symbol include/pmh.h declares, with (restype, argtypes)
_u64, _u32, _i32, _dbl, _vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
_pp = ctypes.POINTER(ctypes.c_void_p)
SIGNATURES = {
    "pmh_init": (_i32, [_u64, _u32, _i32, _pp]),
    "pmh_destroy": (None, [_vp]),
    "pmh_max_m": (_u32, [_i32]),
    "pmh_status_str": (ctypes.c_char_p, [_i32]),
    "pmh_hash_sets": (_i32, [_vp] * 4 + [_u64] + [_vp] * 5),
    "pmh_pminhash_sets": (_i32, [_vp] * 4 + [_u64] + [_vp] * 5),
    "pmh_hash_sets_binary": (_i32, [_vp] * 3 + [_u64] + [_vp] * 5),
    "pmh_update_sets": (_i32, [_vp] * 4 + [_u64] + [_vp] * 6),
    "pmh_bbit_pack": (_i32, [_vp, _u64, _u32, _u32, _vp, _vp]),
    "pmh_bbit_allpairs": (_i32, [_vp, _u32, _u32, _u32, _vp, _vp]),
    "pmh_hash_sets_plain": (_i32, [_vp] * 4 + [_u64] + [_vp] * 5),
    "pmh_hash_sets_noalloc": (_i32, [_vp] * 4 + [_u64] + [_vp] * 5),
    "pmh_hash_sets_bbit": (_i32, [_vp] * 4 + [_u64, _u32] + [_vp] * 6),
    "pmh_hash_sets_graph": (_i32, [_vp] * 4 + [_u64] + [_vp] * 5),
    "pmh_get_status": (_i32, [_vp, _vp]),
    "pmh_timing_begin": (_i32, [_vp, _i32]),
    "pmh_timing_read": (_i32, [_vp, _vp, _i32]),
    "pmh_set_tuning": (_i32, [_vp, _vp]),
    "pmh_set_caps": (_i32, [_vp, _u32, _u32, _u32, _u32]),
    "pmh_get_tuning": (_i32, [_vp, _vp]),
    "pmh_autotune": (_i32, [_vp] * 4 + [_u64, _i32, _vp, _vp]),
    "pmh_tuning_save": (_i32, [_vp, ctypes.c_char_p]),
    "pmh_tuning_load": (_i32, [_vp, ctypes.c_char_p]),
    "pmh_estimate": (_i32, [_vp, _vp, _vp, _vp, _u32, _vp]),
    "pmh_estimate_pairs": (_i32, [_vp, _vp, _vp, _vp, _u32, _u64, _vp, _vp]),
    "pmh_allpairs_counts": (_i32, [_vp, _u32, _u32, _vp, _vp]),
    "pmh_get_table": (_i32, [_vp, _i32, _vp, _u32]),
    "pmh_debug_eval": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _u64, _vp]),
    "pmh_server_create": (_i32, [_vp, _i32, _u64, _u32, _u64, _pp]),
    "pmh_server_submit": (_i32, [_vp, _vp, _vp, _u32, ctypes.POINTER(_u64)]),
    "pmh_server_fetch": (_i32, [_vp, _u64, _vp, _vp, _vp]),
    "pmh_server_replay": (_i32, [_vp, _vp, _vp, _vp, _u64, _vp, _vp, _vp, _vp, ctypes.POINTER(_dbl)]),
    "pmh_server_replay_indexed": (_i32, [_vp, _vp, _vp, _vp, _u64, _vp, _u64, _vp, _vp, _vp, _vp,
                                         ctypes.POINTER(_dbl)]),
    "pmh_server_stats": (_i32, [_vp, _vp]),
    "pmh_server_destroy": (None, [_vp]),
}


class PmhError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = lib().pmh_status_str(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} (status {code})" if what else msg)
        self.code = code


class pmh_tuning(ctypes.Structure):
    _fields_ = [("c0", ctypes.c_double), ("grow", ctypes.c_double), ("max_rounds", ctypes.c_int),
                ("chain_expect", ctypes.c_double), ("lane_budget", ctypes.c_int), ("waves", ctypes.c_int),
                ("kmax_refresh", ctypes.c_int), ("blocks_per_cu", ctypes.c_int), ("mini_expect", ctypes.c_double),
                ("split_log2", ctypes.c_int), ("c0_split", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def lib():
    """Load libpmh.so (built by paper_1911_00675_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_1911_00675_amd.build` first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != PMH_OK:
        raise PmhError(rc, what)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libpmh needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _dptr(t, dtypes, name):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_batch(ids, weights, offsets, out, m):
    """Host-side shape checks the C ABI cannot make: the element arrays cover
    offsets[-1] entries and every output holds num_sets x m entries."""
    num_sets = int(offsets.numel()) - 1
    if num_sets < 0 or offsets.dim() != 1:
        raise ValueError("offsets must be a 1-D tensor of num_sets + 1 entries")
    n = 0
    if num_sets > 0:
        # offsets[-1] costs a device sync; it is remembered on the tensor until
        # the tensor is modified in place (its version counter moves)
        memo = getattr(offsets, "_pmh_total", None)
        if memo is not None and memo[0] == offsets._version:
            n = memo[1]
        else:
            n = int(offsets[-1].item())
            offsets._pmh_total = (offsets._version, n)
    if ids.numel() < n:
        raise ValueError(f"ids holds {ids.numel()} entries, offsets[-1] = {n}")
    if weights is not None and weights.numel() < n:
        raise ValueError(f"weights holds {weights.numel()} entries, offsets[-1] = {n}")
    if out is not None:
        for name in ("idx", "val", "id", "keys"):
            t = getattr(out, name)
            if t is not None and t.numel() != num_sets * m:
                raise ValueError(f"out.{name} holds {t.numel()} entries, expected {num_sets} x {m}")
    return num_sets


def to_device(arr: np.ndarray, device="cuda"):
    """numpy -> device tensor, uint64 carried as int64 bits."""
    torch = _torch()
    if arr.dtype == np.uint64:
        arr = arr.view(np.int64)
    return torch.from_numpy(np.ascontiguousarray(arr)).to(device)


@dataclass
class Signatures:
    idx: object = None   # int32 tensor [S, m], bit pattern of uint32 (0xFFFFFFFF = empty)
    val: object = None   # float64 [S, m]
    id: object = None    # int64 [S, m], bit pattern of uint64
    keys: object = None  # int64 [S, m], bit pattern of uint64
    bbit: object = None  # int64 [S, ceil(m b / 64)]: b-bit reduction (hash_sets(..., bbit=b))


@dataclass
class SetState:
    """Signatures kept across pmh_update_sets calls (device tensors)."""
    keys: object          # int64 [S, m], all ones for a new set
    counts: object        # int32 [S], elements absorbed (bit pattern of uint32)
    id: object = None     # int64 [S, m] or None: ids of the components' elements


class Context:
    """A signature context for (seed, m, variant) on the current device."""

    def __init__(self, seed: int, m: int, variant: int):
        _torch()
        self._c = ctypes.c_void_p()
        _check(lib().pmh_init(seed & KEY_EMPTY, m, variant, ctypes.byref(self._c)), "pmh_init")
        self.seed, self.m, self.variant = seed, m, variant

    def close(self):
        if self._c:
            lib().pmh_destroy(self._c)
            self._c = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ hashing
    def alloc_outputs(self, num_sets: int, outputs=("idx", "val", "id", "keys")) -> Signatures:
        torch = _torch()
        shape = (num_sets, self.m)
        return Signatures(
            idx=torch.empty(shape, dtype=torch.int32, device="cuda") if "idx" in outputs else None,
            val=torch.empty(shape, dtype=torch.float64, device="cuda") if "val" in outputs else None,
            id=torch.empty(shape, dtype=torch.int64, device="cuda") if "id" in outputs else None,
            keys=torch.empty(shape, dtype=torch.int64, device="cuda") if "keys" in outputs else None)

    def hash_sets(self, ids, weights, offsets, out: Signatures | None = None, mode: str = "batched",
                  stream=None, outputs=("idx", "val", "id", "keys"), bbit: int = 0) -> Signatures:
        """Signatures of a CSR batch of device tensors (ids int64/uint64,
        weights float64, offsets int64/uint64 with num_sets+1 entries).
        mode: "batched", "plain", "graph", "noalloc" (ProbMinHash of the
        context's variant; "noalloc" takes its work buffer from the library's
        static array, at most 2^20 sets), "pminhash" (P-MinHash with the context's seed and m) or
        "binary" (the unit-weight specialisation of the context's variant;
        weights must be None)."""
        torch = _torch()
        num_sets = _check_batch(ids, weights, offsets, out, self.m)
        if out is None:
            out = self.alloc_outputs(num_sets, outputs)
        i64 = (torch.int64, torch.uint64)
        if bbit:
            if mode != "batched":
                raise ValueError("the fused b-bit reduction runs in the batched form")
            words = (self.m * bbit + 63) // 64
            if out.bbit is None:
                out.bbit = torch.empty((num_sets, words), dtype=torch.int64, device="cuda")
            elif out.bbit.numel() != num_sets * words:
                raise ValueError(f"out.bbit holds {out.bbit.numel()} entries, expected {num_sets} x {words}")
            rc = lib().pmh_hash_sets_bbit(
                self._c, _dptr(ids, i64, "ids"), _dptr(weights, (torch.float64,), "weights"),
                _dptr(offsets, i64, "offsets"), num_sets, int(bbit), _dptr(out.bbit, (torch.int64,), "bbit"),
                _dptr(out.idx, (torch.int32,), "idx"), _dptr(out.val, (torch.float64,), "val"),
                _dptr(out.id, i64, "id"), _dptr(out.keys, i64, "keys"), _stream_ptr(stream))
            _check(rc, "pmh_hash_sets_bbit")
            return out
        if mode == "binary":
            if weights is not None:
                raise ValueError("binary mode takes no weights")
            rc = lib().pmh_hash_sets_binary(
                self._c, _dptr(ids, i64, "ids"), _dptr(offsets, i64, "offsets"), num_sets,
                _dptr(out.idx, (torch.int32,), "idx"), _dptr(out.val, (torch.float64,), "val"),
                _dptr(out.id, i64, "id"), _dptr(out.keys, i64, "keys"), _stream_ptr(stream))
            _check(rc, "pmh_hash_sets_binary")
            return out
        fn = {"batched": lib().pmh_hash_sets, "plain": lib().pmh_hash_sets_plain,
              "noalloc": lib().pmh_hash_sets_noalloc,
              "graph": lib().pmh_hash_sets_graph, "pminhash": lib().pmh_pminhash_sets}[mode]
        rc = fn(self._c, _dptr(ids, i64, "ids"), _dptr(weights, (torch.float64,), "weights"),
                _dptr(offsets, i64, "offsets"), num_sets,
                _dptr(out.idx, (torch.int32,), "idx"), _dptr(out.val, (torch.float64,), "val"),
                _dptr(out.id, i64, "id"), _dptr(out.keys, i64, "keys"), _stream_ptr(stream))
        _check(rc, f"pmh_hash_sets ({mode})")
        return out

    def new_state(self, num_sets: int, with_id: bool = True) -> SetState:
        """Empty signatures for num_sets sets that grow by update_sets."""
        torch = _torch()
        shape = (num_sets, self.m)
        return SetState(keys=torch.full(shape, -1, dtype=torch.int64, device="cuda"),
                        counts=torch.zeros(num_sets, dtype=torch.int32, device="cuda"),
                        id=torch.zeros(shape, dtype=torch.int64, device="cuda") if with_id else None)

    def update_sets(self, ids, weights, offsets, state: SetState, out: Signatures | None = None,
                    stream=None) -> SetState:
        """Add a CSR batch of new elements (weights None: binary weights) to the
        sets of state, in place; out may receive positions and values."""
        torch = _torch()
        num_sets = _check_batch(ids, weights, offsets, out, self.m)
        if state.keys.shape != (num_sets, self.m) or state.counts.numel() != num_sets:
            raise ValueError("state does not match the batch's sets or the context's m")
        if state.id is not None and state.id.numel() != num_sets * self.m:
            raise ValueError("state.id does not hold num_sets x m entries")
        i64 = (torch.int64, torch.uint64)
        rc = lib().pmh_update_sets(
            self._c, _dptr(ids, i64, "ids"),
            None if weights is None else _dptr(weights, (torch.float64,), "weights"),
            _dptr(offsets, i64, "offsets"), num_sets, _dptr(state.counts, (torch.int32,), "counts"),
            _dptr(state.keys, i64, "keys"), _dptr(out.idx if out else None, (torch.int32,), "idx"),
            _dptr(out.val if out else None, (torch.float64,), "val"), _dptr(state.id, i64, "id"),
            _stream_ptr(stream))
        _check(rc, "pmh_update_sets")
        return state

    def status(self, stream=None) -> int:
        """Synchronize and return (then clear) sticky kernel errors."""
        return lib().pmh_get_status(self._c, _stream_ptr(stream))

    # ------------------------------------------------------------------ timing
    def timing_begin(self, n: int):
        """Record the persistent kernel's duration in the next n batched calls."""
        _check(lib().pmh_timing_begin(self._c, int(n)), "pmh_timing_begin")

    def timing_read(self, n: int) -> np.ndarray:
        out = np.zeros(n, dtype=np.float32)
        _check(lib().pmh_timing_read(self._c, out.ctypes.data_as(ctypes.c_void_p), int(n)), "pmh_timing_read")
        return out

    # ------------------------------------------------------------------ tuning
    def get_tuning(self) -> pmh_tuning:
        t = pmh_tuning()
        _check(lib().pmh_get_tuning(self._c, ctypes.byref(t)), "pmh_get_tuning")
        return t

    def set_tuning(self, **kw):
        t = self.get_tuning()
        for k, v in kw.items():
            setattr(t, k, v)
        _check(lib().pmh_set_tuning(self._c, ctypes.byref(t)), "pmh_set_tuning")

    def set_caps(self, imax: int = 0, te_rounds: int = 32, redraws: int = 8, lemire_floor: int = 0):
        """Loop caps of the streams (see pmh_set_caps); they change results."""
        _check(lib().pmh_set_caps(self._c, int(imax), int(te_rounds), int(redraws), int(lemire_floor)),
               "pmh_set_caps")

    def save_tuning(self, path: str):
        """Store the current tuning under (device arch, CUs, m, variant)."""
        _check(lib().pmh_tuning_save(self._c, os.fsencode(path)), "pmh_tuning_save")

    def load_tuning(self, path: str) -> bool:
        """Apply the stored tuning for this context's key; False if none."""
        rc = lib().pmh_tuning_load(self._c, os.fsencode(path))
        if rc == PMH_ERR_NO_ENTRY:
            return False
        _check(rc, "pmh_tuning_load")
        return True

    def autotune(self, ids, weights, offsets, trials: int = 3, stream=None, cache: str | None = None) -> dict:
        """Time candidate schedules on this batch and keep the fastest.  With
        a cache file, a stored tuning for this device, m and variant is used
        instead, and a new result is stored there."""
        if cache and self.load_tuning(cache):
            return self.get_tuning().as_dict()
        torch = _torch()
        i64 = (torch.int64, torch.uint64)
        best = pmh_tuning()
        rc = lib().pmh_autotune(self._c, _dptr(ids, i64, "ids"), _dptr(weights, (torch.float64,), "weights"),
                                _dptr(offsets, i64, "offsets"), int(offsets.numel()) - 1, trials,
                                _stream_ptr(stream), ctypes.byref(best))
        _check(rc, "pmh_autotune")
        if cache:
            self.save_tuning(cache)
        return best.as_dict()

    # --------------------------------------------------------------- validation
    def table(self, which: int, count: int) -> np.ndarray:
        out = np.zeros(count, dtype=np.float64)
        _check(lib().pmh_get_table(self._c, which, out.ctypes.data_as(ctypes.c_void_p), count), "pmh_get_table")
        return out

    def debug_eval(self, what: int, x: np.ndarray) -> np.ndarray:
        """Evaluate one stream primitive on the device (see pmh_debug_eval)."""
        torch = _torch()
        n = int(x.size)
        uses_u = 3 <= what <= 7 or what >= 9
        out_u = what in (4, 6, 7, 9, 10, 11, 12)
        xin = to_device(x.astype(np.uint64) if uses_u else x.astype(np.float64))
        o = torch.empty(n, dtype=torch.int64 if out_u else torch.float64, device="cuda")
        rc = lib().pmh_debug_eval(self._c, what, None if uses_u else ctypes.c_void_p(xin.data_ptr()),
                                  ctypes.c_void_p(xin.data_ptr()) if uses_u else None,
                                  None if out_u else ctypes.c_void_p(o.data_ptr()),
                                  ctypes.c_void_p(o.data_ptr()) if out_u else None, n, _stream_ptr(None))
        _check(rc, "pmh_debug_eval")
        torch.cuda.synchronize()
        r = o.cpu().numpy()
        return r.view(np.uint64) if out_u else r


def estimate(idA, idxA, idB, idxB) -> float:
    """Host estimator of eq. (3) for one pair (numpy arrays)."""
    idA = np.ascontiguousarray(idA).view(np.uint64) if np.asarray(idA).dtype == np.int64 else np.ascontiguousarray(idA, dtype=np.uint64)
    idB = np.ascontiguousarray(idB).view(np.uint64) if np.asarray(idB).dtype == np.int64 else np.ascontiguousarray(idB, dtype=np.uint64)
    idxA = np.ascontiguousarray(idxA).view(np.uint32)
    idxB = np.ascontiguousarray(idxB).view(np.uint32)
    out = ctypes.c_double()
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    _check(lib().pmh_estimate(vp(idA), vp(idxA), vp(idB), vp(idxB), idA.size, ctypes.byref(out)), "pmh_estimate")
    return out.value


def estimate_pairs(idA, idxA, idB, idxB, stream=None):
    """Equal-component counts for [pairs, m] device tensors; returns int32 [pairs]."""
    torch = _torch()
    pairs, m = idA.shape
    counts = torch.empty(pairs, dtype=torch.int32, device="cuda")
    i64 = (torch.int64, torch.uint64)
    rc = lib().pmh_estimate_pairs(_dptr(idA, i64, "idA"), _dptr(idxA, (torch.int32,), "idxA"),
                                  _dptr(idB, i64, "idB"), _dptr(idxB, (torch.int32,), "idxB"), m, pairs,
                                  _dptr(counts, (torch.int32,), "counts"), _stream_ptr(stream))
    _check(rc, "pmh_estimate_pairs")
    return counts


def allpairs_counts(fp, stream=None):
    """All-pairs equal-component counts of k fingerprint signatures fp [k, m]
    (int32 device tensor, 0 = empty); returns int16 [k, k] (bits of uint16)."""
    torch = _torch()
    k, m = fp.shape
    counts = torch.empty((k, k), dtype=torch.int16, device="cuda")
    rc = lib().pmh_allpairs_counts(_dptr(fp, (torch.int32,), "fp"), k, m, _dptr(counts, (torch.int16,), "counts"),
                                   _stream_ptr(stream))
    _check(rc, "pmh_allpairs_counts")
    return counts


def bbit_pack(ids, b: int, stream=None):
    """b-bit reduction (Sec. 1.3) of signatures given by their element ids
    [num_sigs, m] (int64 device tensor, 0 = empty): int64 [num_sigs, words]."""
    torch = _torch()
    S, m = ids.shape
    out = torch.empty((S, (m * b + 63) // 64), dtype=torch.int64, device="cuda")
    rc = lib().pmh_bbit_pack(_dptr(ids, (torch.int64, torch.uint64), "ids"), S, m, b,
                             _dptr(out, (torch.int64,), "out"), _stream_ptr(stream))
    _check(rc, "pmh_bbit_pack")
    return out


def bbit_allpairs(sig, m: int, b: int, stream=None):
    """All-pairs equal-field counts of packed b-bit signatures [k, words]:
    int16 [k, k] (bits of uint16)."""
    torch = _torch()
    k = sig.shape[0]
    counts = torch.empty((k, k), dtype=torch.int16, device="cuda")
    rc = lib().pmh_bbit_allpairs(_dptr(sig, (torch.int64,), "sig"), k, m, b, _dptr(counts, (torch.int16,), "counts"),
                                 _stream_ptr(stream))
    _check(rc, "pmh_bbit_allpairs")
    return counts


class Server:
    """Continuous-batching server (see pmh_server_create)."""

    def __init__(self, ctx: Context, slots: int = 4, slot_elems: int = 1 << 22, slot_sets: int = 4096,
                 hbm_budget: int = 0):
        self.ctx = ctx
        self._s = ctypes.c_void_p()
        _check(lib().pmh_server_create(ctx._c, slots, slot_elems, slot_sets, hbm_budget, ctypes.byref(self._s)),
               "pmh_server_create")

    def submit(self, ids: np.ndarray, weights: np.ndarray) -> int:
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        w = np.ascontiguousarray(weights, dtype=np.float64)
        t = ctypes.c_uint64()
        _check(lib().pmh_server_submit(self._s, ids.ctypes.data_as(ctypes.c_void_p),
                                       w.ctypes.data_as(ctypes.c_void_p), ids.size, ctypes.byref(t)),
               "pmh_server_submit")
        return t.value

    def fetch(self, ticket: int):
        """(idx uint32[m], val float64[m], id uint64[m]) or None if not ready."""
        m = self.ctx.m
        idx = np.zeros(m, dtype=np.uint32)
        val = np.zeros(m, dtype=np.float64)
        idv = np.zeros(m, dtype=np.uint64)
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        rc = lib().pmh_server_fetch(self._s, ticket, vp(idx), vp(val), vp(idv))
        if rc == PMH_ERR_NOT_READY:
            return None
        _check(rc, "pmh_server_fetch")
        return idx, val, idv

    def replay(self, ids, weights, offsets, arrival):
        """Open-loop replay of CSR host requests at the given arrival times (s).
        Returns (latency[num] s, idx[num, m], id[num, m], wall s)."""
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        w = np.ascontiguousarray(weights, dtype=np.float64)
        off = np.ascontiguousarray(offsets, dtype=np.uint64)
        arr = np.ascontiguousarray(arrival, dtype=np.float64)
        num = off.size - 1
        m = self.ctx.m
        lat = np.zeros(num, dtype=np.float64)
        idx = np.zeros((num, m), dtype=np.uint32)
        idv = np.zeros((num, m), dtype=np.uint64)
        wall = ctypes.c_double()
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(lib().pmh_server_replay(self._s, vp(ids), vp(w), vp(off), num, vp(arr), vp(lat), vp(idx), vp(idv),
                                       ctypes.byref(wall)), "pmh_server_replay")
        return lat, idx, idv, wall.value

    def replay_indexed(self, ids, weights, offsets, order, arrival):
        """Open-loop replay of requests drawn from a CSR pool of host requests
        (request r is pool entry order[r]).  Returns (latency[num] s, wall s);
        no signatures are copied back."""
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        w = np.ascontiguousarray(weights, dtype=np.float64)
        off = np.ascontiguousarray(offsets, dtype=np.uint64)
        order = np.ascontiguousarray(order, dtype=np.uint64)
        arr = np.ascontiguousarray(arrival, dtype=np.float64)
        if order.size != arr.size:
            raise ValueError("order and arrival differ in length")
        lat = np.zeros(arr.size, dtype=np.float64)
        wall = ctypes.c_double()
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(lib().pmh_server_replay_indexed(self._s, vp(ids), vp(w), vp(off), off.size - 1, vp(order),
                                               order.size, vp(arr), vp(lat), None, None, ctypes.byref(wall)),
               "pmh_server_replay_indexed")
        return lat, wall.value

    def stats(self) -> dict:
        o = np.zeros(8, dtype=np.uint64)
        _check(lib().pmh_server_stats(self._s, o.ctypes.data_as(ctypes.c_void_p)), "pmh_server_stats")
        return dict(batches=int(o[0]), done=int(o[1]), max_batch=int(o[2]), max_busy_slots=int(o[3]),
                    waited=int(o[4]), max_launch_us=int(o[5]), max_finish_us=int(o[6]), max_iter_us=int(o[7]))

    def close(self):
        if self._s:
            lib().pmh_server_destroy(self._s)
            self._s = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
