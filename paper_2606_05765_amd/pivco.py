"""Python binding of the gfx950 PivCo-Huffman library (``libpivco.so``).

Argument marshalling only: every step of encoding and decoding runs in the
library's HIP kernels.  PyTorch provides device memory (``torch.uint8`` CUDA
tensors on ROCm) and the current HIP stream.  The functions carry the names
of the C entry points in ``include/pivco.h``.  If the library is missing
this module raises at import time of ``lib()``; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpivco.so")

OK, E_ARG, E_CAPACITY, E_CORRUPT, E_UNSUPPORTED, E_DEVICE, E_BUDGET = 0, -1, -2, -3, -4, -5, -6
_NAMES = {0: "OK", -1: "E_ARG", -2: "E_CAPACITY", -3: "E_CORRUPT", -4: "E_UNSUPPORTED",
          -5: "E_DEVICE", -6: "E_BUDGET"}


class PivcoError(RuntimeError):
    def __init__(self, code, what=""):
        super().__init__(f"{what}: {_NAMES.get(code, code)} ({code})")
        self.code = code


class Tree(C.Structure):
    _fields_ = [("code_len", C.c_uint8 * 256)]


class EncodeOpts(C.Structure):
    _fields_ = [("block_size", C.c_uint32), ("max_len", C.c_uint32), ("ans_mode", C.c_uint32),
                ("rans_chunk_log2", C.c_uint32), ("tree", C.POINTER(Tree)),
                ("tree_shape", C.c_uint32), ("reserved", C.c_uint32)]


class Job(C.Structure):
    _fields_ = [("d_in", C.c_void_p), ("in_len", C.c_uint64), ("d_out", C.c_void_p),
                ("out_cap", C.c_uint64)]


class Tune(C.Structure):
    _fields_ = [("merge_variant", C.c_uint32), ("merge_grid", C.c_uint32),
                ("rans_grid", C.c_uint32), ("grid_mode", C.c_uint32)]

    def as_dict(self):
        return {"merge_variant": self.merge_variant, "merge_grid": self.merge_grid,
                "rans_grid": self.rans_grid, "grid_mode": self.grid_mode}


class ServerOpts(C.Structure):
    _fields_ = [("mem_budget", C.c_uint64), ("slots", C.c_uint32), ("max_batch", C.c_uint32),
                ("max_blocks", C.c_uint32), ("merge_variant", C.c_uint32),
                ("max_scratch_words", C.c_uint64), ("keep_outputs", C.c_uint32),
                ("max_tiles", C.c_uint32)]


class Request(C.Structure):
    _fields_ = [("arrival_s", C.c_double), ("id", C.c_uint32), ("reserved", C.c_uint32)]


class RequestResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("reserved", C.c_uint32), ("d_out", C.c_void_p),
                ("n_out", C.c_uint64), ("t_admit", C.c_double), ("t_done", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("wall_s", C.c_double), ("bytes_decoded", C.c_uint64),
                ("peak_pool_bytes", C.c_uint64), ("batches", C.c_uint64), ("max_batch", C.c_uint64),
                ("max_busy_slots", C.c_uint64)]


_lib = None


def lib():
    """Load libpivco.so (built by ``paper_2606_05765_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2606_05765_amd/build.py "
                              "(the HIP library is the only implementation)")
        L = C.CDLL(LIB_PATH)
        vp, u32, u64, i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32
        u64p = C.POINTER(C.c_uint64)
        u32p = C.POINTER(C.c_uint32)
        sigs = {
            "pivco_build_tree": (i32, [u64p, u32, C.POINTER(Tree)]),
            "pivco_encode_bound": (u64, [u64, C.POINTER(EncodeOpts)]),
            "pivco_encode_workspace": (u64, [u64, C.POINTER(EncodeOpts)]),
            "pivco_encode": (i32, [vp, u64, vp, u64, u64p, C.POINTER(EncodeOpts), vp, u64, vp]),
            "pivco_encode_async": (i32, [vp, u64, vp, u64, vp, vp, C.POINTER(EncodeOpts), vp, u64, vp]),
            "pivco_stream_info": (i32, [vp, u64, u64p, u32p, u32p, u64p]),
            "pivco_decode_workspace": (u64, [C.POINTER(Job), u32, vp]),
            "pivco_decode_batch": (i32, [C.POINTER(Job), u32, vp, vp, u64, vp]),
            "pivco_decode": (i32, [vp, u64, vp, u64, vp, vp, u64, vp]),
            "pivco_decode_plain": (i32, [C.POINTER(Job), u32, vp, vp, u64, vp]),
            "pivco_decode_topdown": (i32, [C.POINTER(Job), u32, vp, vp, u64, vp]),
            "pivco_decode_noalloc": (i32, [vp, u64, vp, u64, vp, vp]),
            "pivco_merge_variants": (u32, []),
            "pivco_merge_variant_name": (C.c_char_p, [u32]),
            "pivco_batch_plan_create": (i32, [C.POINTER(Job), u32, vp, vp, u64, C.POINTER(Tune),
                                              vp, C.POINTER(vp)]),
            "pivco_batch_plan_launch": (i32, [vp, vp]),
            "pivco_batch_plan_launch_timed": (i32, [vp, vp, vp, vp]),
            "pivco_batch_plan_destroy": (None, [vp]),
            "pivco_autotune": (i32, [C.POINTER(Job), u32, vp, vp, u64, vp, C.POINTER(Tune)]),
            "pivco_autotune_cache_clear": (None, []),
            "pivco_golomb_encode_bound": (u64, [u64, u32]),
            "pivco_golomb_encode_workspace": (u64, [u64, u32]),
            "pivco_golomb_encode": (i32, [vp, u64, u32, vp, u64, u64p, vp, u64, vp]),
            "pivco_golomb_decode_workspace": (u64, [C.POINTER(Job), u32, vp]),
            "pivco_golomb_decode": (i32, [C.POINTER(Job), u32, vp, vp, u64, vp]),
            "pivco_strerror": (C.c_char_p, [i32]),
            "pivco_server_create": (i32, [C.POINTER(ServerOpts), C.POINTER(vp)]),
            "pivco_server_destroy": (None, [vp]),
            "pivco_server_workspace_bytes": (u64, [vp]),
            "pivco_server_register": (i32, [vp, vp, u64, u32p]),
            "pivco_server_run": (i32, [vp, C.POINTER(Request), u32, vp, u64,
                                       C.POINTER(RequestResult), C.POINTER(ServerStats)]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        raise PivcoError(rc, what)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_u8(t):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.uint8 and t.is_contiguous()):
        raise TypeError("expected a contiguous torch.uint8 CUDA tensor")
    return t


# ---------------------------------------------------------------------------
# tree
# ---------------------------------------------------------------------------

def pivco_build_tree(counts, max_len=11):
    c = np.ascontiguousarray(np.asarray(counts, dtype=np.uint64).reshape(256))
    t = Tree()
    _check(lib().pivco_build_tree(c.ctypes.data_as(C.POINTER(C.c_uint64)), max_len, C.byref(t)),
           "pivco_build_tree")
    return np.frombuffer(bytes(t.code_len), dtype=np.uint8).copy()


# ---------------------------------------------------------------------------
# encode
# ---------------------------------------------------------------------------

def _opts(block_size, max_len, ans_mode, chunk_log2, tree, flat=False):
    o = EncodeOpts(block_size, max_len, ans_mode, chunk_log2, None, 1 if flat else 0, 0)
    keep = None
    if tree is not None:
        keep = Tree()
        keep.code_len[:] = [int(x) for x in np.asarray(tree, dtype=np.uint8).reshape(256)]
        o.tree = C.pointer(keep)
    return o, keep


def pivco_encode_bound(n, block_size, max_len=11, ans_mode=0, chunk_log2=16, flat=False):
    o, _ = _opts(block_size, max_len, ans_mode, chunk_log2, None, flat)
    return int(lib().pivco_encode_bound(n, C.byref(o)))


def pivco_encode(data, block_size, max_len=11, ans_mode=0, chunk_log2=16, tree=None, flat=False):
    """Encode a uint8 CUDA tensor; returns the stream as a uint8 CUDA tensor
    (v1 with canonical trees, or v2 with flat-subtree trees when flat=True)."""
    data = _dev_u8(data)
    n = data.numel()
    o, keep = _opts(block_size, max_len, ans_mode, chunk_log2, tree, flat)
    cap = int(lib().pivco_encode_bound(n, C.byref(o)))
    wsb = int(lib().pivco_encode_workspace(n, C.byref(o)))
    if cap == 0:
        raise PivcoError(E_ARG, "pivco_encode_bound")
    out = torch.empty(cap, dtype=torch.uint8, device=data.device)
    ws = torch.empty(max(wsb, 256), dtype=torch.uint8, device=data.device)
    olen = C.c_uint64(0)
    _check(lib().pivco_encode(C.c_void_p(data.data_ptr() if n else 0), n, C.c_void_p(out.data_ptr()),
                              cap, C.byref(olen), C.byref(o), C.c_void_p(ws.data_ptr()), ws.numel(),
                              _stream()), "pivco_encode")
    del keep
    return out[:olen.value].clone()


def pivco_encode_async(data, out, out_len, status, ws, block_size, max_len=11, ans_mode=0, chunk_log2=16,
                       tree=None, flat=False):
    """Enqueue an encode on the current stream without waiting: the stream
    goes to out (a uint8 CUDA tensor of at least pivco_encode_bound bytes),
    its length to out_len (a one-element int64 CUDA tensor) and the status to
    status (a one-element int32 CUDA tensor); ws is a uint8 CUDA tensor of at
    least pivco_encode_workspace bytes."""
    data = _dev_u8(data)
    out = _dev_u8(out)
    ws = _dev_u8(ws)
    if not (out_len.is_cuda and out_len.dtype == torch.int64 and status.is_cuda and status.dtype == torch.int32):
        raise TypeError("out_len: an int64 CUDA tensor, status: an int32 CUDA tensor")
    n = data.numel()
    o, keep = _opts(block_size, max_len, ans_mode, chunk_log2, tree, flat)
    _check(lib().pivco_encode_async(C.c_void_p(data.data_ptr() if n else 0), n, C.c_void_p(out.data_ptr()),
                                    out.numel(), C.c_void_p(out_len.data_ptr()), C.c_void_p(status.data_ptr()),
                                    C.byref(o), C.c_void_p(ws.data_ptr()), ws.numel(), _stream()),
           "pivco_encode_async")
    del keep


def pivco_encode_workspace(n, block_size, max_len=11, ans_mode=0, chunk_log2=16, flat=False):
    o, _ = _opts(block_size, max_len, ans_mode, chunk_log2, None, flat)
    return int(lib().pivco_encode_workspace(n, C.byref(o)))


# ---------------------------------------------------------------------------
# decode
# ---------------------------------------------------------------------------

def pivco_stream_info(stream):
    h = np.frombuffer(bytes(stream[:48].cpu().numpy().tobytes()) if isinstance(stream, torch.Tensor)
                      else bytes(stream)[:48], dtype=np.uint8).copy()
    n = C.c_uint64(0); nb = C.c_uint32(0); bs = C.c_uint32(0); aw = C.c_uint64(0)
    _check(lib().pivco_stream_info(h.ctypes.data_as(C.c_void_p), h.size, C.byref(n), C.byref(nb),
                                   C.byref(bs), C.byref(aw)), "pivco_stream_info")
    return {"n_total": n.value, "n_blocks": nb.value, "block_size": bs.value, "ans_words": aw.value}


def _jobs(streams, outs):
    arr = (Job * max(len(streams), 1))()
    for i, (s, o) in enumerate(zip(streams, outs)):
        arr[i].d_in = s.data_ptr() if s.numel() else None
        arr[i].in_len = s.numel()
        arr[i].d_out = o.data_ptr() if o.numel() else None
        arr[i].out_cap = o.numel()
    return arr


def _alloc_outs(streams, outs):
    if outs is not None:
        return [_dev_u8(o) for o in outs]
    res = []
    for s in streams:
        n = pivco_stream_info(s)["n_total"]
        res.append(torch.empty(n, dtype=torch.uint8, device=s.device))
    return res


def pivco_decode_workspace(streams, outs):
    jobs = _jobs(streams, outs)
    w = int(lib().pivco_decode_workspace(jobs, len(streams), _stream()))
    if w == 0 and len(streams):
        raise PivcoError(E_ARG, "pivco_decode_workspace")
    return w


class Workspace:
    """A reusable device workspace sized for a set of jobs."""

    def __init__(self, nbytes, device="cuda"):
        self.tensor = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)

    @property
    def ptr(self):
        return C.c_void_p(self.tensor.data_ptr())

    @property
    def nbytes(self):
        return self.tensor.numel()


def pivco_decode_batch(streams, outs=None, ws=None, plain=False, entry="pivco_decode_batch"):
    """Decode a list of streams in one batched launch.  Returns (outs, status)
    where status is a CPU int32 numpy array (one pivco status per job)."""
    streams = [_dev_u8(s) for s in streams]
    outs = _alloc_outs(streams, outs)
    jobs = _jobs(streams, outs)
    if ws is None:
        ws = Workspace(pivco_decode_workspace(streams, outs))
    status = torch.zeros(max(len(streams), 1), dtype=torch.int32, device="cuda")
    name = "pivco_decode_plain" if plain else entry
    _check(getattr(lib(), name)(jobs, len(streams), C.c_void_p(status.data_ptr()), ws.ptr, ws.nbytes,
                                _stream()), name)
    return outs, status[:len(streams)].cpu().numpy()


def pivco_decode_topdown(streams, outs=None, ws=None):
    """The top-down (partition/scatter) decode of the same streams."""
    return pivco_decode_batch(streams, outs, ws=ws, entry="pivco_decode_topdown")


def pivco_decode(stream, out=None, ws=None):
    outs, st = pivco_decode_batch([stream], None if out is None else [out], ws=ws)
    return outs[0], int(st[0])


NOALLOC_SCRATCH_BYTES = 32 << 20


def pivco_decode_noalloc(stream, out, status):
    """pivco_decode with the library's fixed device scratch: no workspace,
    no allocation (out and status are caller tensors: uint8 and int32)."""
    stream = _dev_u8(stream)
    out = _dev_u8(out)
    if not (status.is_cuda and status.dtype == torch.int32 and status.numel() >= 1):
        raise TypeError("status: an int32 CUDA tensor")
    _check(lib().pivco_decode_noalloc(C.c_void_p(stream.data_ptr()), stream.numel(),
                                      C.c_void_p(out.data_ptr() if out.numel() else 0), out.numel(),
                                      C.c_void_p(status.data_ptr()), _stream()),
           "pivco_decode_noalloc")


def pivco_decode_plain(streams, outs=None, ws=None):
    return pivco_decode_batch(streams, outs, ws=ws, plain=True)


def pivco_merge_variants():
    n = int(lib().pivco_merge_variants())
    return [lib().pivco_merge_variant_name(i).decode() for i in range(n)]


def pivco_autotune(streams, outs, ws=None):
    streams = [_dev_u8(s) for s in streams]
    jobs = _jobs(streams, outs)
    if ws is None:
        ws = Workspace(pivco_decode_workspace(streams, outs))
    status = torch.zeros(max(len(streams), 1), dtype=torch.int32, device="cuda")
    t = Tune()
    _check(lib().pivco_autotune(jobs, len(streams), C.c_void_p(status.data_ptr()), ws.ptr,
                                ws.nbytes, _stream(), C.byref(t)), "pivco_autotune")
    return t


def pivco_autotune_cache_clear():
    lib().pivco_autotune_cache_clear()


class BatchPlan:
    """pivco_batch_plan_*: job table uploaded once, decode captured in a HIP
    graph, each launch() replays it on the current stream."""

    def __init__(self, streams, outs, tune=None, ws=None):
        self.streams = [_dev_u8(s) for s in streams]
        self.outs = [_dev_u8(o) for o in outs]
        self.jobs = _jobs(self.streams, self.outs)
        self.ws = ws if ws is not None else Workspace(pivco_decode_workspace(self.streams, self.outs))
        self.status = torch.zeros(max(len(streams), 1), dtype=torch.int32, device="cuda")
        self.handle = C.c_void_p()
        self.tune = tune
        _check(lib().pivco_batch_plan_create(self.jobs, len(self.streams),
                                             C.c_void_p(self.status.data_ptr()), self.ws.ptr,
                                             self.ws.nbytes,
                                             C.byref(tune) if tune is not None else None,
                                             _stream(), C.byref(self.handle)),
               "pivco_batch_plan_create")

    def launch(self):
        _check(lib().pivco_batch_plan_launch(self.handle, _stream()), "pivco_batch_plan_launch")

    def launch_timed(self, ev_begin, ev_end):
        """Eager launch with HIP events recorded around the merge kernel
        (torch.cuda.Event objects, recorded on the current stream)."""
        _check(lib().pivco_batch_plan_launch_timed(self.handle, _stream(),
                                                   C.c_void_p(ev_begin.cuda_event),
                                                   C.c_void_p(ev_end.cuda_event)),
               "pivco_batch_plan_launch_timed")

    def statuses(self):
        return self.status[:len(self.streams)].cpu().numpy()

    def close(self):
        if self.handle:
            lib().pivco_batch_plan_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """pivco_server_*: continuous-batching decode of resident streams."""

    def __init__(self, mem_budget, slots=4, max_batch=64, max_blocks=1 << 16,
                 max_scratch_words=1 << 24, merge_variant=0, keep_outputs=False, max_tiles=0):
        o = ServerOpts(int(mem_budget), slots, max_batch, max_blocks, merge_variant,
                       max_scratch_words, 1 if keep_outputs else 0, max_tiles)
        self.handle = C.c_void_p()
        _check(lib().pivco_server_create(C.byref(o), C.byref(self.handle)), "pivco_server_create")
        self.streams = []

    def register(self, stream):
        stream = _dev_u8(stream)
        rid = C.c_uint32(0)
        _check(lib().pivco_server_register(self.handle, C.c_void_p(stream.data_ptr()),
                                           stream.numel(), C.byref(rid)), "pivco_server_register")
        self.streams.append(stream)
        return rid.value

    def workspace_bytes(self):
        return int(lib().pivco_server_workspace_bytes(self.handle))

    def run(self, arrivals, ids, pool):
        """Replay (arrival_s, id) pairs; returns (results list of dicts, stats dict)."""
        n = len(ids)
        reqs = (Request * max(n, 1))()
        for i, (a, r) in enumerate(zip(arrivals, ids)):
            reqs[i].arrival_s = float(a)
            reqs[i].id = int(r)
        res = (RequestResult * max(n, 1))()
        st = ServerStats()
        _check(lib().pivco_server_run(self.handle, reqs, n, C.c_void_p(pool.data_ptr()), pool.numel(),
                                      res, C.byref(st)), "pivco_server_run")
        out = [{"status": res[i].status, "d_out": res[i].d_out, "n_out": res[i].n_out,
                "t_admit": res[i].t_admit, "t_done": res[i].t_done, "arrival": float(arrivals[i])}
               for i in range(n)]
        return out, {"wall_s": st.wall_s, "bytes_decoded": st.bytes_decoded,
                     "peak_pool_bytes": st.peak_pool_bytes, "batches": st.batches,
                     "max_batch": st.max_batch, "max_busy_slots": st.max_busy_slots}

    def close(self):
        if self.handle:
            lib().pivco_server_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def view_output(pool, d_out, n):
    """The decoded bytes of one served request as a tensor view into pool."""
    off = int(d_out) - pool.data_ptr()
    return pool[off:off + n]


# ---------------------------------------------------------------------------
# PivCo-Golomb (App. G): unary codes in the pivoted list-of-bitmaps layout
# ---------------------------------------------------------------------------

def pivco_golomb_encode(data, block_size):
    """Encode a uint8 CUDA tensor of values; returns the stream (CUDA tensor)."""
    data = _dev_u8(data)
    n = data.numel()
    cap = int(lib().pivco_golomb_encode_bound(n, block_size))
    wsb = int(lib().pivco_golomb_encode_workspace(n, block_size))
    if cap == 0:
        raise PivcoError(E_ARG, "pivco_golomb_encode_bound")
    out = torch.empty(cap, dtype=torch.uint8, device=data.device)
    ws = torch.empty(max(wsb, 256), dtype=torch.uint8, device=data.device)
    olen = C.c_uint64(0)
    _check(lib().pivco_golomb_encode(C.c_void_p(data.data_ptr() if n else 0), n, block_size,
                                     C.c_void_p(out.data_ptr()), cap, C.byref(olen),
                                     C.c_void_p(ws.data_ptr()), ws.numel(), _stream()),
           "pivco_golomb_encode")
    return out[:olen.value].clone()


def pivco_golomb_decode(streams, outs=None):
    """Decode PivCo-Golomb streams in one launch; returns (outs, status)."""
    streams = [_dev_u8(s) for s in streams]
    if outs is None:
        outs = []
        for s in streams:
            n = int.from_bytes(bytes(s[8:16].cpu().numpy().tobytes()), "little")
            outs.append(torch.empty(n, dtype=torch.uint8, device=s.device))
    outs = [_dev_u8(o) for o in outs]
    jobs = _jobs(streams, outs)
    wsb = int(lib().pivco_golomb_decode_workspace(jobs, len(streams), _stream()))
    ws = Workspace(wsb)
    status = torch.zeros(max(len(streams), 1), dtype=torch.int32, device="cuda")
    _check(lib().pivco_golomb_decode(jobs, len(streams), C.c_void_p(status.data_ptr()), ws.ptr,
                                     ws.nbytes, _stream()), "pivco_golomb_decode")
    return outs, status[:len(streams)].cpu().numpy()
