"""Python binding of libdqmc (ctypes; argument marshalling only).

Every function here forwards to the C ABI of the same name declared in
``include/dqmc.h``; all computation happens in the HIP kernels of
``libdqmc.so``.  Device buffers are torch tensors on a ROCm device (torch is
used for device memory and streams only); they are passed by ``data_ptr()``
together with the current torch stream.  There is no fallback: if the library
cannot be loaded or the GPU is unavailable, calls raise.

dtypes: truth tables and states are ``torch.int32`` tensors holding the
uint32 words bit for bit; lists, counts and dense bitmaps are ``torch.int64``
tensors holding uint64 values.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdqmc.so")

DQMC_OK, DQMC_EINVAL, DQMC_ENOMEM, DQMC_EDEVICE, DQMC_ESCRATCH, DQMC_EIO = 0, -1, -2, -3, -4, -5
DQMC_MAX_N = 25

_lib = None
_lock = threading.Lock()


class DqmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("dqmc error %d: %s" % (code, msg))
        self.code = code


class dqmc_pass_record(ctypes.Structure):
    _fields_ = [
        ("pass_", ctypes.c_char * 40),
        ("n", ctypes.c_int32),
        ("list_bytes_per_prime", ctypes.c_int32),
        ("ms", ctypes.c_float),
        ("model_bytes", ctypes.c_double),
    ]


DQMC_MAX_RECORDS = 64
DQMC_MAX_PLAN_TRIALS = 64
DQMC_NEGATE = 1
DQMC_SPARSE_MAX_N = 31
DQMC_SLICED_MAX_N = 30
DQMC_SLICED_MAX_T = 8
DQMC_SLICED_MAX_STATES = 16


class dqmc_result(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("count", ctypes.c_uint64),
        ("listed", ctypes.c_uint64),
        ("state", ctypes.c_void_p),
        ("list", ctypes.c_void_p),
        ("t_submit", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
    ]


class dqmc_job(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("tt", ctypes.c_void_p),
        ("state", ctypes.c_void_p),
        ("list", ctypes.c_void_p),
        ("list_cap", ctypes.c_uint64),
        ("count", ctypes.c_void_p),
    ]


class dqmc_batch_trial(ctypes.Structure):
    _fields_ = [("col_cap", ctypes.c_int32), ("order", ctypes.c_int32), ("ms", ctypes.c_float)]


class dqmc_plan_trial(ctypes.Structure):
    _fields_ = [("ngroups", ctypes.c_int32), ("sizes", ctypes.c_int32 * DQMC_MAX_N), ("ms", ctypes.c_float)]


def load():
    """Load libdqmc.so (building it first only if it does not exist)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            from . import build as _build

            _build.build()
        # torch ships its own HIP runtime under the same soname as the
        # system one.  Loaded first, it also serves libdqmc.so, so that the
        # library and the tensors it is given share one runtime; loaded
        # after the library, a second runtime would come up beside it.
        import torch  # noqa: F401

        lib = ctypes.CDLL(LIB_PATH)
        u64, i32, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
        sig = {
            "dqmc_create": (i32, [i32, ctypes.POINTER(vp)]),
            "dqmc_destroy": (None, [vp]),
            "dqmc_last_error": (ctypes.c_char_p, [vp]),
            "dqmc_num_cubes": (u64, [i32]),
            "dqmc_tt_words": (u64, [i32]),
            "dqmc_state_words": (u64, [i32]),
            "dqmc_dense_words": (u64, [i32]),
            "dqmc_implicants": (i32, [vp, i32, vp, vp, vp]),
            "dqmc_primes": (i32, [vp, i32, vp, vp, vp, u64, vp, vp]),
            "dqmc_implicants_ex": (i32, [vp, i32, vp, ctypes.c_uint32, vp, vp]),
            "dqmc_sparse_workspace_bytes": (u64, [i32, u64, u64]),
            "dqmc_sparse_primes": (i32, [vp, i32, vp, vp, u64, vp, vp, u64, ctypes.POINTER(ctypes.c_uint64), vp]),
            "dqmc_primes_ex": (i32, [vp, i32, vp, ctypes.c_uint32, vp, vp, u64, vp, vp]),
            "dqmc_primes_noalloc": (i32, [i32, vp, vp, vp, u64, vp, vp]),
            "dqmc_extract": (i32, [vp, i32, vp, vp, u64, vp, vp]),
            "dqmc_primes_sliced": (i32, [vp, i32, i32, vp, ctypes.c_uint32, vp, vp, vp, u64, vp, vp]),
            "dqmc_primes_sliced_multi": (i32, [vp, i32, i32, vp, ctypes.c_uint32, vp, ctypes.POINTER(vp), i32, vp,
                                               u64, vp, vp]),
            "dqmc_bitmap_to_dense": (i32, [vp, i32, vp, vp, vp]),
            "dqmc_primes_batch": (i32, [vp, vp, ctypes.c_int32, vp]),
            "dqmc_profile": (i32, [vp, i32]),
            "dqmc_batch_create": (i32, [vp, vp, ctypes.c_int32, ctypes.POINTER(vp)]),
            "dqmc_batch_config": (i32, [vp, ctypes.c_int32, ctypes.c_int32]),
            "dqmc_batch_run": (i32, [vp, vp]),
            "dqmc_batch_destroy": (None, [vp]),
            "dqmc_set_plan": (i32, [vp, i32, ctypes.POINTER(ctypes.c_int32), i32]),
            "dqmc_hash_words": (i32, [vp, vp, u64, vp, vp]),
            "dqmc_server_create": (i32, [i32, u64, ctypes.c_int32, ctypes.POINTER(vp)]),
            "dqmc_server_submit": (i32, [vp, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_uint64)]),
            "dqmc_server_poll": (i32, [vp, ctypes.c_uint64, ctypes.POINTER(dqmc_result)]),
            "dqmc_server_wait": (i32, [vp, ctypes.c_uint64, ctypes.POINTER(dqmc_result)]),
            "dqmc_server_release": (i32, [vp, ctypes.c_uint64]),
            "dqmc_server_read": (ctypes.c_int64, [vp, ctypes.c_uint64, vp, ctypes.c_uint64]),
            "dqmc_server_destroy": (None, [vp]),
            "dqmc_get_plan": (i32, [vp, i32, ctypes.POINTER(ctypes.c_int32), i32]),
            "dqmc_set_split": (i32, [vp, i32, i32]),
            "dqmc_get_split": (i32, [vp, i32]),
            "dqmc_tune_save": (i32, [vp, ctypes.c_char_p]),
            "dqmc_flag_units": (i32, [vp, ctypes.POINTER(ctypes.c_uint64)]),
            "dqmc_tune_load": (i32, [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)]),
            "dqmc_profile_read": (i32, [vp, ctypes.POINTER(dqmc_pass_record), i32]),
            "dqmc_batch_autotune": (i32, [vp, ctypes.c_int32, vp, ctypes.POINTER(dqmc_batch_trial), ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32)]),
            "dqmc_plan_autotune": (i32, [vp, i32, vp, vp, vp, ctypes.c_int32, ctypes.c_int32, vp,
                                         ctypes.POINTER(dqmc_plan_trial), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
        return lib


# ----------------------------------------------------------------------------
# sizes (pure host functions)

def dqmc_num_cubes(n: int) -> int:
    return int(load().dqmc_num_cubes(n))


def dqmc_tt_words(n: int) -> int:
    return int(load().dqmc_tt_words(n))


def dqmc_state_words(n: int) -> int:
    return int(load().dqmc_state_words(n))


def dqmc_dense_words(n: int) -> int:
    return int(load().dqmc_dense_words(n))


# ----------------------------------------------------------------------------
# marshalling helpers

def _ptr(t, what, dtype, min_numel):
    import torch

    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % what)
    if t.device.type != "cuda":
        raise ValueError("%s must be a device tensor" % what)
    if t.dtype != dtype:
        raise TypeError("%s must have dtype %s (got %s)" % (what, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if t.numel() < min_numel:
        raise ValueError("%s has %d elements, needs %d" % (what, t.numel(), min_numel))
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _check(ctx, rc):
    if rc != DQMC_OK:
        msg = load().dqmc_last_error(ctx)
        raise DqmcError(rc, msg.decode() if msg else "")


# ----------------------------------------------------------------------------
# the C ABI, one function each

def dqmc_create(device: int = 0) -> ctypes.c_void_p:
    import torch

    if not torch.cuda.is_available():
        raise DqmcError(DQMC_EDEVICE, "no ROCm device visible")
    out = ctypes.c_void_p()
    rc = load().dqmc_create(device, ctypes.byref(out))
    if rc != DQMC_OK:
        raise DqmcError(rc, "dqmc_create(%d) failed" % device)
    return out


def dqmc_destroy(ctx) -> None:
    load().dqmc_destroy(ctx)


def dqmc_last_error(ctx) -> str:
    m = load().dqmc_last_error(ctx)
    return m.decode() if m else ""


def dqmc_implicants(ctx, n, tt, state, stream=None) -> None:
    import torch

    _check(ctx, load().dqmc_implicants(
        ctx, n, _ptr(tt, "tt", torch.int32, dqmc_tt_words(n)),
        _ptr(state, "state", torch.int32, dqmc_state_words(n)), _stream(stream)))


def dqmc_primes(ctx, n, tt, state, lst, list_cap, count, stream=None) -> None:
    import torch

    cap = 0 if lst is None else int(list_cap)
    _check(ctx, load().dqmc_primes(
        ctx, n, _ptr(tt, "tt", torch.int32, dqmc_tt_words(n)),
        _ptr(state, "state", torch.int32, dqmc_state_words(n)),
        _ptr(lst, "list", torch.int64, cap), cap,
        _ptr(count, "count", torch.int64, 1), _stream(stream)))


def dqmc_primes_noalloc(n, tt, state, lst, list_cap, count, stream=None) -> None:
    """No context: the library's fixed device scratch, on the current device."""
    import torch

    cap = 0 if lst is None else int(list_cap)
    rc = load().dqmc_primes_noalloc(
        n, _ptr(tt, "tt", torch.int32, dqmc_tt_words(n)),
        _ptr(state, "state", torch.int32, dqmc_state_words(n)),
        _ptr(lst, "list", torch.int64, cap), cap,
        _ptr(count, "count", torch.int64, 1), _stream(stream))
    if rc != DQMC_OK:
        raise DqmcError(rc, "dqmc_primes_noalloc(n=%d) failed" % n)


def dqmc_implicants_ex(ctx, n, tt, flags, state, stream=None) -> None:
    import torch

    _check(ctx, load().dqmc_implicants_ex(ctx, n, _ptr(tt, "tt", torch.int32, dqmc_tt_words(n)), int(flags),
                                          _ptr(state, "state", torch.int32, dqmc_state_words(n)), _stream(stream)))


def dqmc_primes_ex(ctx, n, tt, flags, state, lst, list_cap, count, stream=None) -> None:
    import torch

    cap = 0 if lst is None else int(list_cap)
    _check(ctx, load().dqmc_primes_ex(ctx, n, _ptr(tt, "tt", torch.int32, dqmc_tt_words(n)), int(flags),
                                      _ptr(state, "state", torch.int32, dqmc_state_words(n)),
                                      _ptr(lst, "list", torch.int64, cap), cap,
                                      _ptr(count, "count", torch.int64, 1), _stream(stream)))


def dqmc_sparse_workspace_bytes(n: int, max_level: int, max_primes: int) -> int:
    return int(load().dqmc_sparse_workspace_bytes(n, int(max_level), int(max_primes)))


def dqmc_sparse_primes(ctx, n, tt, lst, list_cap, count, work, stream=None):
    """Sparse path (see include/dqmc.h).  `work` is a uint8 device tensor.
    Returns (status, largest level, primes seen); status DQMC_ENOMEM means
    the workspace was too small (nothing written), other errors raise."""
    import torch

    if not isinstance(work, torch.Tensor) or work.device.type != "cuda" or work.dtype != torch.uint8:
        raise TypeError("work must be a uint8 device tensor")
    need = (ctypes.c_uint64 * 2)()
    cap = 0 if lst is None else int(list_cap)
    nw = max(1, (1 << n) // 32) if 0 <= n <= DQMC_SPARSE_MAX_N else 1  # the library rejects other n
    rc = load().dqmc_sparse_primes(ctx, n, _ptr(tt, "tt", torch.int32, nw), _ptr(lst, "list", torch.int64, cap), cap,
                                   _ptr(count, "count", torch.int64, 1), ctypes.c_void_p(work.data_ptr()),
                                   work.numel(), need, _stream(stream))
    if rc != DQMC_ENOMEM:
        _check(ctx, rc)
    return rc, int(need[0]), int(need[1])


def dqmc_primes_sliced(ctx, n, t, tt, flags, o_state, m_state, lst, list_cap, count, stream=None) -> None:
    """Sliced path (see include/dqmc.h): o_state and m_state each hold
    dqmc_state_words(n - t) words."""
    import torch

    cap = 0 if lst is None else int(list_cap)
    ok = 1 <= t <= DQMC_SLICED_MAX_T and t <= n <= DQMC_SLICED_MAX_N and n - t <= DQMC_MAX_N
    nw = max(1, (1 << n) // 32) if ok else 1  # the library rejects other n, t
    sw = dqmc_state_words(n - t) if ok else 1
    _check(ctx, load().dqmc_primes_sliced(
        ctx, n, t, _ptr(tt, "tt", torch.int32, nw), int(flags), _ptr(o_state, "o_state", torch.int32, sw),
        _ptr(m_state, "m_state", torch.int32, sw), _ptr(lst, "list", torch.int64, cap), cap,
        _ptr(count, "count", torch.int64, 1), _stream(stream)))


def dqmc_primes_sliced_multi(ctx, n, t, tt, flags, o_state, m_states, lst, list_cap, count, stream=None) -> None:
    """Sliced path with several implicant states (see include/dqmc.h)."""
    import torch

    cap = 0 if lst is None else int(list_cap)
    ok = 1 <= t <= DQMC_SLICED_MAX_T and t <= n <= DQMC_SLICED_MAX_N and n - t <= DQMC_MAX_N
    nw = max(1, (1 << n) // 32) if ok else 1  # the library rejects other n, t
    sw = dqmc_state_words(n - t) if ok else 1
    ptrs = [_ptr(m, "m_states[%d]" % i, torch.int32, sw) for i, m in enumerate(m_states)]
    arr = (ctypes.c_void_p * max(1, len(ptrs)))(*[p.value for p in ptrs])
    _check(ctx, load().dqmc_primes_sliced_multi(
        ctx, n, t, _ptr(tt, "tt", torch.int32, nw), int(flags), _ptr(o_state, "o_state", torch.int32, sw),
        arr, len(ptrs), _ptr(lst, "list", torch.int64, cap), cap, _ptr(count, "count", torch.int64, 1),
        _stream(stream)))


def dqmc_extract(ctx, n, state, lst, list_cap, count, stream=None) -> None:
    import torch

    cap = 0 if lst is None else int(list_cap)
    _check(ctx, load().dqmc_extract(
        ctx, n, _ptr(state, "state", torch.int32, dqmc_state_words(n)),
        _ptr(lst, "list", torch.int64, cap), cap,
        _ptr(count, "count", torch.int64, 1), _stream(stream)))


def dqmc_bitmap_to_dense(ctx, n, state, dense, stream=None) -> None:
    import torch

    _check(ctx, load().dqmc_bitmap_to_dense(
        ctx, n, _ptr(state, "state", torch.int32, dqmc_state_words(n)),
        _ptr(dense, "dense", torch.int64, dqmc_dense_words(n)), _stream(stream)))


def _job_array(jobs):
    import torch

    arr = (dqmc_job * max(1, len(jobs)))()
    for i, j in enumerate(jobs):
        n = int(j["n"])
        # sizes are checked for the n a batch accepts; other jobs are passed
        # through for the library to reject
        nn = n if 0 <= n <= 16 else 0
        lst = j.get("list")
        cap = 0 if lst is None else int(j.get("list_cap", lst.numel()))
        arr[i].n = n
        arr[i].status = 0
        arr[i].tt = _ptr(j["tt"], "tt", torch.int32, dqmc_tt_words(nn)) if j.get("tt") is not None else None
        arr[i].state = _ptr(j["state"], "state", torch.int32, dqmc_state_words(nn)) if j.get("state") is not None else None
        arr[i].list = _ptr(lst, "list", torch.int64, cap)
        arr[i].list_cap = cap
        arr[i].count = _ptr(j["count"], "count", torch.int64, 1) if j.get("count") is not None else None
    return arr


def job_table(jobs, device=None):
    """The device-resident dqmc_job array for a list of job dicts (keys n, tt,
    state, list (or None), list_cap, count; device tensors), as a uint8
    device tensor.  Invalid jobs are passed through for the library to
    reject."""
    import torch

    arr = _job_array(jobs)
    host = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8)
    if device is None:
        device = next((j[k].device for j in jobs for k in ("state", "tt", "count")
                       if j.get(k) is not None), torch.device("cuda"))
    return host.to(device)


def job_status(table, njobs: int) -> list:
    """The status fields of a device job table (waits for the copy)."""
    import numpy as np

    raw = table.cpu().numpy().view(np.uint8)
    rec = np.frombuffer(raw.tobytes(), dtype=np.int32).reshape(-1, ctypes.sizeof(dqmc_job) // 4)
    return [int(x) for x in rec[:njobs, 1]]


def dqmc_primes_batch(ctx, jobs, stream=None, njobs=None):
    """dqmc_primes_batch.  ``jobs`` is a device job table (from job_table;
    then only enqueued, and None is returned) or a list of job dicts (then the
    table is built, the call is enqueued, the stream is waited for, and the
    per-job status codes are returned)."""
    import torch

    if isinstance(jobs, torch.Tensor):
        k = int(njobs) if njobs is not None else jobs.numel() // ctypes.sizeof(dqmc_job)
        _check(ctx, load().dqmc_primes_batch(ctx, ctypes.c_void_p(jobs.data_ptr()), k, _stream(stream)))
        return None
    table = job_table(jobs)
    _check(ctx, load().dqmc_primes_batch(ctx, ctypes.c_void_p(table.data_ptr()), len(jobs), _stream(stream)))
    torch.cuda.synchronize()
    return job_status(table, len(jobs))


class Batch:
    """A batch plan (dqmc_batch_create / config / run / destroy) over a device
    job table built from ``jobs``.  The job tensors must stay alive while the
    plan is used; the statuses are written by every run."""

    def __init__(self, ctx, jobs):
        self.ctx = ctx
        self._jobs = jobs  # keep the tensors alive
        self.table = job_table(jobs)
        self.njobs = len(jobs)
        out = ctypes.c_void_p()
        _check(ctx, load().dqmc_batch_create(ctx, ctypes.c_void_p(self.table.data_ptr()), len(jobs),
                                             ctypes.byref(out)))
        self.plan = out

    @property
    def status(self) -> list:
        """Per-job status codes of the last run (waits for the device)."""
        import torch

        torch.cuda.synchronize()
        return job_status(self.table, self.njobs)

    def config(self, col_cap: int = 0, order: int = 0):
        _check(self.ctx, load().dqmc_batch_config(self.plan, col_cap, order))

    def run(self, stream=None):
        _check(self.ctx, load().dqmc_batch_run(self.plan, _stream(stream)))

    def autotune(self, reps: int = 3, stream=None) -> list:
        """dqmc_batch_autotune: time the column-cap/order candidates, keep the
        fastest; returns the trials as dicts (col_cap, order, ms)."""
        arr = (dqmc_batch_trial * 16)()
        k = ctypes.c_int32(0)
        _check(self.ctx, load().dqmc_batch_autotune(self.plan, reps, _stream(stream), arr, 16, ctypes.byref(k)))
        return [dict(col_cap=arr[i].col_cap, order=arr[i].order, ms=float(arr[i].ms))
                for i in range(min(k.value, 16))]

    def close(self):
        if self.plan is not None:
            load().dqmc_batch_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dqmc_hash_words(ctx, words, nwords: int, out, stream=None) -> None:
    """Order-dependent hash of nwords device words (a tensor or a raw device
    address) into the int64 device tensor `out`."""
    import torch

    addr = ctypes.c_void_p(words.data_ptr() if isinstance(words, torch.Tensor) else int(words))
    _check(ctx, load().dqmc_hash_words(ctx, addr, int(nwords), _ptr(out, "out", torch.int64, 1), _stream(stream)))


def _result_dict(r):
    return dict(n=r.n, status=r.status, count=int(r.count), listed=int(r.listed), state=r.state, list=r.list,
                t_submit=r.t_submit, t_admit=r.t_admit, t_done=r.t_done)


class Server:
    """The request loop of dqmc_server_* (admission by memory footprint,
    continuous batching, results kept on the device until released)."""

    def __init__(self, device: int = 0, budget: int = 0, slots: int = 4):
        import torch

        if not torch.cuda.is_available():
            raise DqmcError(DQMC_EDEVICE, "no ROCm device visible")
        out = ctypes.c_void_p()
        rc = load().dqmc_server_create(device, int(budget), int(slots), ctypes.byref(out))
        if rc != DQMC_OK:
            raise DqmcError(rc, "dqmc_server_create failed")
        self.srv = out

    def submit(self, n: int, tt) -> int:
        import numpy as np

        a = np.ascontiguousarray(tt, dtype=np.uint32)
        if a.size < dqmc_tt_words(n) if 0 <= n <= DQMC_MAX_N else False:
            raise ValueError("truth table too short")
        jid = ctypes.c_uint64()
        rc = load().dqmc_server_submit(self.srv, int(n), a.ctypes.data, ctypes.byref(jid))
        if rc != DQMC_OK:
            raise DqmcError(rc, "submit failed")
        return int(jid.value)

    def poll(self, jid: int):
        r = dqmc_result()
        rc = load().dqmc_server_poll(self.srv, jid, ctypes.byref(r))
        if rc < 0:
            raise DqmcError(rc, "poll: unknown job %d" % jid)
        return _result_dict(r) if rc == 1 else None

    def wait(self, jid: int):
        r = dqmc_result()
        rc = load().dqmc_server_wait(self.srv, jid, ctypes.byref(r))
        if rc != DQMC_OK:
            raise DqmcError(rc, "wait: unknown job %d" % jid)
        return _result_dict(r)

    def read(self, jid: int, cap: int):
        import numpy as np

        out = np.zeros(max(1, int(cap)), dtype=np.uint64)
        k = load().dqmc_server_read(self.srv, jid, out.ctypes.data, int(cap))
        if k < 0:
            raise DqmcError(int(k), "read failed")
        return out[:k]

    def release(self, jid: int):
        rc = load().dqmc_server_release(self.srv, jid)
        if rc != DQMC_OK:
            raise DqmcError(rc, "release failed")

    def close(self):
        if self.srv is not None:
            load().dqmc_server_destroy(self.srv)
            self.srv = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def dqmc_set_plan(ctx, n: int, sizes) -> None:
    """Group sizes of digits 13..n for this context ([] = default plan)."""
    arr = (ctypes.c_int32 * max(1, len(sizes)))(*[int(x) for x in sizes])
    _check(ctx, load().dqmc_set_plan(ctx, n, arr, len(sizes)))


def dqmc_get_plan(ctx, n: int) -> list:
    arr = (ctypes.c_int32 * 32)()
    k = load().dqmc_get_plan(ctx, n, arr, 32)
    if k < 0:
        _check(ctx, k)
    return [int(arr[i]) for i in range(k)]


def dqmc_plan_autotune(ctx, n: int, tt, state, count, extra_groups: int = 0, reps: int = 2, stream=None) -> list:
    """Time the pass plans for n (see include/dqmc.h), set the fastest on
    the context; returns the trials as dicts (sizes, ms)."""
    import torch

    cap = DQMC_MAX_PLAN_TRIALS + 1  # the group plans and the top-digit split
    arr = (dqmc_plan_trial * cap)()
    k = ctypes.c_int32(0)
    rc = load().dqmc_plan_autotune(ctx, n, _ptr(tt, "tt", torch.int32, dqmc_tt_words(n)),
                                   _ptr(state, "state", torch.int32, dqmc_state_words(n)),
                                   _ptr(count, "count", torch.int64, 1), int(extra_groups), int(reps),
                                   _stream(stream), arr, cap, ctypes.byref(k))
    _check(ctx, rc)
    return [dict(sizes=[int(arr[i].sizes[g]) for g in range(arr[i].ngroups)], ms=float(arr[i].ms),
                 split=arr[i].ngroups == 0) for i in range(min(k.value, cap))]


def dqmc_set_split(ctx, n: int, mode: int) -> None:
    """Top-digit split of dqmc_primes for n: 1 on, 0 off, -1 default."""
    _check(ctx, load().dqmc_set_split(ctx, n, int(mode)))


def dqmc_get_split(ctx, n: int) -> bool:
    return load().dqmc_get_split(ctx, n) == 1


def dqmc_flag_units(ctx) -> dict:
    """Bytes of the data-dependent passes of the last flagged n = 24 call."""
    u = (ctypes.c_uint64 * 4)()
    _check(ctx, load().dqmc_flag_units(ctx, u))
    return {"reduce13_rows_bytes": int(u[0]), "final_runs_bytes": int(u[1]), "final_store_bytes": int(u[2]),
            "used": bool(u[3])}


def dqmc_tune_save(ctx, path: str) -> None:
    """Write the context's non-default plans and split modes (JSON, keyed by
    the device architecture and n)."""
    _check(ctx, load().dqmc_tune_save(ctx, os.fsencode(path)))


def dqmc_tune_load(ctx, path: str) -> int:
    """Apply a tuning file written for this device's architecture; returns
    the number of entries applied (0 for a file of another architecture)."""
    k = ctypes.c_int32(0)
    _check(ctx, load().dqmc_tune_load(ctx, os.fsencode(path), ctypes.byref(k)))
    return int(k.value)


def dqmc_profile(ctx, enable: bool) -> None:
    _check(ctx, load().dqmc_profile(ctx, 1 if enable else 0))


def dqmc_profile_read(ctx) -> list:
    """Records of the passes enqueued since profiling was enabled or last
    read: dicts with pass, n, ms, model_bytes, list_bytes_per_prime."""
    arr = (dqmc_pass_record * DQMC_MAX_RECORDS)()
    k = load().dqmc_profile_read(ctx, arr, DQMC_MAX_RECORDS)
    if k < 0:
        _check(ctx, k)
    return [dict(pass_name=arr[i].pass_.decode(), n=arr[i].n, ms=float(arr[i].ms),
                 model_bytes=float(arr[i].model_bytes), list_bytes_per_prime=arr[i].list_bytes_per_prime)
            for i in range(k)]


# ----------------------------------------------------------------------------
# convenience wrapper

class Context:
    """Owns a dqmc context on one device and allocates result tensors."""

    def __init__(self, device: int = 0):
        import torch

        self.device = device
        self.torch_device = torch.device("cuda", device)
        self.ctx = dqmc_create(device)

    def close(self):
        if self.ctx is not None:
            dqmc_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def tt_to_device(self, tt_u32):
        """Host uint32 numpy truth table -> device int32 tensor."""
        import numpy as np
        import torch

        a = np.ascontiguousarray(tt_u32, dtype=np.uint32).view(np.int32)
        return torch.from_numpy(a.copy()).to(self.torch_device)

    def new_state(self, n):
        import torch

        return torch.empty(dqmc_state_words(n), dtype=torch.int32, device=self.torch_device)

    def implicants(self, n, tt, state=None, stream=None):
        state = self.new_state(n) if state is None else state
        dqmc_implicants(self.ctx, n, tt, state, stream)
        return state

    def primes(self, n, tt, state=None, list_cap=None, stream=None, flags=0):
        """(state, list, count) device tensors; with list_cap None the list
        has room for every possible prime of this call's count (two passes).
        flags=DQMC_NEGATE: the primes of the complement of the table."""
        import torch

        state = self.new_state(n) if state is None else state
        count = torch.zeros(1, dtype=torch.int64, device=self.torch_device)
        if list_cap is None:
            dqmc_primes_ex(self.ctx, n, tt, flags, state, None, 0, count, stream)
            cap = int(count.item())
            lst = torch.empty(max(cap, 1), dtype=torch.int64, device=self.torch_device)
            dqmc_extract(self.ctx, n, state, lst, cap, count, stream)
            return state, lst[:cap], count
        lst = torch.empty(max(int(list_cap), 1), dtype=torch.int64, device=self.torch_device)
        dqmc_primes_ex(self.ctx, n, tt, flags, state, lst, list_cap, count, stream)
        return state, lst, count

    def sparse_primes(self, n, tt, work_bytes=None, stream=None):
        """(list, count) of the sparse path; the workspace grows as needed
        (one retry with the sizes the first attempt reports)."""
        import torch

        count = torch.zeros(1, dtype=torch.int64, device=self.torch_device)
        if work_bytes is None:
            work_bytes = 256 << 20
        lv = npr = 0
        for _ in range(8):
            work = torch.empty(int(work_bytes), dtype=torch.uint8, device=self.torch_device)
            rc, lv2, npr2 = dqmc_sparse_primes(self.ctx, n, tt, None, 0, count, work, stream)
            if rc == DQMC_OK:
                break
            # a failed attempt only saw the levels up to the one that overflowed
            lv, npr = max(lv, lv2) * 2, max(npr, npr2, 1) * 2
            work_bytes = max(dqmc_sparse_workspace_bytes(n, lv, npr), 2 * int(work_bytes))
            del work
        else:
            raise DqmcError(DQMC_ENOMEM, "sparse workspace still too small")
        c = int(count.item())
        lst = torch.empty(max(c, 1), dtype=torch.int64, device=self.torch_device)
        rc, _, _ = dqmc_sparse_primes(self.ctx, n, tt, lst, c, count, work, stream)
        if rc != DQMC_OK:
            raise DqmcError(rc, "sparse path failed on the second run")
        return lst[:c], count

    def sliced_primes(self, n, t, tt, list_cap=None, flags=0, states=None, n_m=1, stream=None):
        """(list, count) of the sliced path with slices of n - t variables.
        states: (o_state, m_state, ...), else allocated here with n_m
        implicant states.  With list_cap None a count-only call sizes the list
        first (the work runs twice)."""
        import torch

        if states is None:
            states = [self.new_state(n - t) for _ in range(1 + n_m)]
        count = torch.zeros(1, dtype=torch.int64, device=self.torch_device)
        o, ms = states[0], list(states[1:])
        if list_cap is None:
            dqmc_primes_sliced_multi(self.ctx, n, t, tt, flags, o, ms, None, 0, count, stream)
            list_cap = int(count.item())
        lst = torch.empty(max(int(list_cap), 1), dtype=torch.int64, device=self.torch_device)
        dqmc_primes_sliced_multi(self.ctx, n, t, tt, flags, o, ms, lst, list_cap, count, stream)
        return lst[:int(list_cap)], count

    def extract(self, n, state, list_cap, stream=None):
        import torch

        count = torch.zeros(1, dtype=torch.int64, device=self.torch_device)
        lst = torch.empty(max(int(list_cap), 1), dtype=torch.int64, device=self.torch_device)
        dqmc_extract(self.ctx, n, state, lst, list_cap, count, stream)
        return lst, count

    def to_dense(self, n, state, stream=None):
        import torch

        dense = torch.empty(dqmc_dense_words(n), dtype=torch.int64, device=self.torch_device)
        dqmc_bitmap_to_dense(self.ctx, n, state, dense, stream)
        return dense
