"""Python handle over one partition of the C ABI (argument marshalling only;
every step of the simulation runs in the library's HIP kernels)."""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import FIELDS, W_BF16, W_F32, Desc, Ptype, check, load


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _stream_handle(stream):
    """hipStream_t of a torch stream (or an int), None -> legacy default."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _check_device(tensor, n: int) -> None:
    import torch
    if not (tensor.is_cuda and tensor.dtype == torch.float32 and tensor.is_contiguous() and tensor.numel() >= n):
        raise ValueError(f"need a contiguous float32 device tensor of at least {n} elements")


def enkf_analysis(X, Y, y_obs, r_var, inflation: float = 1.0, seed: int = 0, it: int = 0,
                  lo: float = -3.0e38, hi: float = 3.0e38, stream=None) -> None:
    """One ensemble Kalman analysis on the GPU, in place on X.  X [M, P],
    Y [M, O], y_obs [O]: contiguous float32 device tensors; r_var: host
    observation-error variances [O]."""
    M, P = X.shape
    O = Y.shape[1]
    _check_device(X, M * P)
    _check_device(Y, M * O)
    _check_device(y_obs, O)
    if Y.shape[0] != M:
        raise ValueError("X and Y need one row per member")
    r = np.ascontiguousarray(r_var, dtype=np.float32).reshape(O)
    check(load().dtb_enkf_analysis(M, P, O, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                   ctypes.c_void_p(y_obs.data_ptr()), _ptr(r), float(inflation), int(seed),
                                   int(it), float(lo), float(hi), _stream_handle(stream)))


class Net:
    """One partition on the GPU.

    ``network`` is a ``netgen.Network``-like object (attributes n, n_regions,
    max_delay, row_ptr, col, w, delay, is_inh, region, ptype, ptypes, V0, E,
    tau_ms, dt_ms, bg_lambda, bg_w, seed, member).
    """

    def __init__(self, network, wtype: str = "f32", record_steps: int = 1024, stream=None, _members=None,
                 bundle_syn: int = 0, unroll: int = 0, fuse: int = 0, events: int = 0):
        lib = load()
        self._lib = lib
        h = ctypes.c_void_p()
        if _members is None:
            d, keep = _make_desc(network, wtype, record_steps, bundle_syn, unroll, fuse, events)
            check(lib.dtb_create(ctypes.byref(d), _stream_handle(stream), ctypes.byref(h)))
        else:
            descs = (Desc * len(_members))()
            keep = []
            for m, nw in enumerate(_members):
                d, k = _make_desc(nw, wtype, record_steps, bundle_syn, unroll, fuse, events)
                descs[m] = d
                keep.append(k)
            check(lib.dtb_create_batch(descs, len(_members), _stream_handle(stream), ctypes.byref(h)))
            del descs
        del keep
        self._h = h
        nm = ctypes.c_int32(0)
        check(lib.dtb_batch_info(h, ctypes.byref(nm), None, None, 0))
        self.n_members = nm.value
        noff = np.zeros(nm.value + 1, dtype=np.int64)
        roff = np.zeros(nm.value + 1, dtype=np.int32)
        check(lib.dtb_batch_info(h, None, _ptr(noff), _ptr(roff), nm.value))
        self.neuron_offset, self.region_offset = noff, roff
        self.n = int(noff[-1])
        self.n_regions = int(roff[-1])
        self.words = int(lib.dtb_bitmap_words(self.n))
        self.record_steps = int(record_steps)
        self.n_remote = 0
        self.t = 0

    @classmethod
    def batch(cls, members, wtype: str = "f32", record_steps: int = 1024, stream=None, bundle_syn: int = 0,
              unroll: int = 0, fuse: int = 0, events: int = 0) -> "Net":
        """One handle advancing several independent networks together."""
        return cls(None, wtype=wtype, record_steps=record_steps, stream=stream, _members=list(members),
                   bundle_syn=bundle_syn, unroll=unroll, fuse=fuse, events=events)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.dtb_destroy(h)
        self._h = None

    def __del__(self):
        self.close()

    # ------------------------------------------------------------ stepping
    def step(self, n_steps: int = 1) -> None:
        st = self._lib.dtb_step(self._h, int(n_steps))
        if st != 0:
            # the library may have taken some of the steps before failing
            steps = ctypes.c_int64(self.t)
            if self._lib.dtb_read_counters(self._h, ctypes.byref(steps), None, None, None) == 0:
                self.t = int(steps.value)
            check(st)
        self.t += int(n_steps)

    def run(self, n_steps: int) -> None:
        """n_steps steps as one captured HIP graph (replayed on later calls)."""
        check(self._lib.dtb_run(self._h, int(n_steps)))
        self.t += int(n_steps)

    def set_gains(self, gains) -> None:
        g = np.ascontiguousarray(gains, dtype=np.float32).reshape(self.n_regions, 4)
        check(self._lib.dtb_set_gains(self._h, _ptr(g), 0))

    def set_gains_from(self, tensor) -> None:
        """Gains from a device tensor (float32 [n_regions, 4], contiguous)."""
        _check_device(tensor, self.n_regions * 4)
        check(self._lib.dtb_set_gains(self._h, ctypes.c_void_p(tensor.data_ptr()), 1))

    def bold_into(self, tensor) -> None:
        """BOLD of every population into a device tensor (float32 [n_regions])."""
        _check_device(tensor, self.n_regions)
        check(self._lib.dtb_read_bold(self._h, ctypes.c_void_p(tensor.data_ptr()), None, 1))

    def bold(self, state: bool = False):
        y = np.zeros(self.n_regions, dtype=np.float32)
        st = np.zeros((self.n_regions, 4), dtype=np.float32) if state else None
        check(self._lib.dtb_read_bold(self._h, _ptr(y), None if st is None else _ptr(st), 0))
        return (y, st) if state else y

    def reset(self) -> None:
        check(self._lib.dtb_reset(self._h))
        self.t = 0

    def set_background(self, bg_lambda: float, bg_w: float) -> None:
        check(self._lib.dtb_set_background(self._h, float(bg_lambda), float(bg_w)))

    def set_background_ou(self, mu: float, sigma: float, tau_ms: float) -> None:
        """Ornstein-Uhlenbeck background current instead of the Poisson drive."""
        check(self._lib.dtb_set_background_ou(self._h, float(mu), float(sigma), float(tau_ms)))

    def force(self, raster: np.ndarray) -> None:
        """Queue teacher-forced spikes: raster [n_steps, n] of 0/1."""
        r = np.ascontiguousarray(raster, dtype=np.uint8).reshape(-1, self.n)
        bits = pack_bits(r, self.words)
        check(self._lib.dtb_force_spikes(self._h, _ptr(bits), int(r.shape[0])))

    def set_remote_block(self, block) -> None:
        """Second in-edge block from n_remote neurons of other partitions
        (J_inter); their spikes are replayed with push_remote."""
        keep = [np.ascontiguousarray(block.row_ptr, dtype=np.int64), np.ascontiguousarray(block.col, dtype=np.int32),
                np.ascontiguousarray(block.w, dtype=np.float32), np.ascontiguousarray(block.delay, dtype=np.uint8),
                np.ascontiguousarray(block.is_inh, dtype=np.uint8)]
        if keep[0].shape != (self.n + 1,) or keep[4].shape != (int(block.n_remote),):
            raise ValueError("remote block shapes do not match n / n_remote")
        check(self._lib.dtb_set_remote_block(self._h, int(block.n_remote), int(keep[0][-1]),
                                             *[_ptr(a) for a in keep]))
        self.n_remote = int(block.n_remote)
        self.remote_words = (self.n_remote + 31) // 32

    def push_remote(self, raster: np.ndarray) -> None:
        """Queue the remote spikes of the next steps: raster [n_steps, n_remote] of 0/1."""
        r = np.ascontiguousarray(raster, dtype=np.uint8).reshape(-1, self.n_remote)
        self.push_remote_bits(pack_bits(r, self.remote_words))

    def push_remote_bits(self, bits: np.ndarray) -> None:
        """Queue packed remote spikes [n_steps, ceil(n_remote / 32)] uint32."""
        b = np.ascontiguousarray(bits, dtype=np.uint32)
        b = b.reshape(-1, self.remote_words) if self.n_remote else b.reshape(1, -1)
        check(self._lib.dtb_push_remote_spikes(self._h, _ptr(b), int(b.shape[0])))

    def save(self) -> bytes:
        """The handle's dynamic state (checkpoint) as bytes."""
        used = ctypes.c_size_t(0)
        check(self._lib.dtb_save(self._h, None, 0, ctypes.byref(used)))
        buf = np.zeros(used.value, dtype=np.uint8)
        check(self._lib.dtb_save(self._h, _ptr(buf), buf.size, ctypes.byref(used)))
        return buf.tobytes()

    def load(self, state: bytes) -> None:
        """Resume from a state returned by save() on a handle of the same shape."""
        buf = np.frombuffer(state, dtype=np.uint8)
        check(self._lib.dtb_load(self._h, ctypes.c_void_p(buf.ctypes.data), buf.size))
        steps = ctypes.c_int64(0)
        check(self._lib.dtb_read_counters(self._h, ctypes.byref(steps), None, None, None))
        self.t = int(steps.value)

    def set_timing(self, enable: bool) -> None:
        check(self._lib.dtb_set_timing(self._h, 1 if enable else 0))

    def read_timing(self) -> dict:
        """Summed kernel durations (ms) and launch counts since the last read."""
        ms = np.zeros(9, dtype=np.float64)
        n = np.zeros(9, dtype=np.int64)
        check(self._lib.dtb_read_timing(self._h, _ptr(ms), _ptr(n)))
        names = ("neuron_update", "compact", "gather", "sums", "finalize", "remote_gather", "events",
                 "spike_runs", "background")
        return {k: {"ms": float(ms[q]), "launches": int(n[q])} for q, k in enumerate(names)}

    def sync(self) -> None:
        check(self._lib.dtb_sync(self._h))

    # ---------------------------------------------------------------- reads
    def spikes_bits(self, t0: int, t1: int) -> np.ndarray:
        out = np.zeros((max(0, t1 - t0), self.words), dtype=np.uint32)
        check(self._lib.dtb_read_spikes(self._h, int(t0), int(t1), _ptr(out), 0))
        return out

    def raster(self, t0: int, t1: int) -> np.ndarray:
        """uint8 [t1-t0, n] spike raster of the recorded steps."""
        return unpack_bits(self.spikes_bits(t0, t1), self.n)

    def spike_ids(self, t=None, cap=None, with_count=False):
        """Ascending ids of the neurons that spiked in step t (default: the
        most recent step); with_count also returns the total (may exceed cap)."""
        t = self.t - 1 if t is None else int(t)
        cap = self.n if cap is None else int(cap)
        ids = np.zeros(max(cap, 1), dtype=np.int32)
        cnt = ctypes.c_int64(0)
        check(self._lib.dtb_read_spike_ids(self._h, t, _ptr(ids), cap, ctypes.byref(cnt)))
        out = ids[:min(cap, cnt.value)].copy()
        return (out, int(cnt.value)) if with_count else out

    def state(self, field: str) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.float32)
        check(self._lib.dtb_read_state(self._h, FIELDS[field], _ptr(out), 0))
        return out

    def state_into(self, field: str, tensor) -> None:
        """Read a state field into a device tensor (float32, >= n elements)."""
        check(self._lib.dtb_read_state(self._h, FIELDS[field], ctypes.c_void_p(tensor.data_ptr()), 1))

    def region_counts(self, t0: int, t1: int) -> np.ndarray:
        out = np.zeros((max(0, t1 - t0), self.n_regions), dtype=np.int32)
        check(self._lib.dtb_read_region_counts(self._h, int(t0), int(t1), _ptr(out)))
        return out

    def region_rates(self, t0: int, t1: int) -> np.ndarray:
        out = np.zeros(self.n_regions, dtype=np.float32)
        check(self._lib.dtb_read_region_rates(self._h, int(t0), int(t1), _ptr(out)))
        return out

    def step_events(self, t0: int, t1: int):
        er = np.zeros(max(0, t1 - t0), dtype=np.int64)
        eb = np.zeros(max(0, t1 - t0), dtype=np.int64)
        check(self._lib.dtb_read_step_events(self._h, int(t0), int(t1), _ptr(er), _ptr(eb)))
        return er, eb

    def counters(self) -> dict:
        v = [ctypes.c_int64(0) for _ in range(4)]
        check(self._lib.dtb_read_counters(self._h, *[ctypes.byref(x) for x in v]))
        return {"steps": v[0].value, "spikes": v[1].value, "ev_rec": v[2].value, "ev_bg": v[3].value}


def _make_desc(nw, wtype, record_steps, bundle_syn=0, unroll=0, fuse=0, events=0):
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return _ptr(a)

    d = Desc()
    d.n = int(nw.n)
    d.n_regions = int(nw.n_regions)
    d.max_delay = int(nw.max_delay)
    pt = np.ascontiguousarray(nw.ptypes, dtype=np.float32).reshape(-1, 11)
    d.n_ptypes = int(pt.shape[0])
    d.member = int(getattr(nw, "member", 0))
    d.nnz = int(nw.row_ptr[-1])
    d.row_ptr = arr(nw.row_ptr, np.int64)
    d.col = arr(nw.col, np.int32)
    d.w = arr(nw.w, np.float32)
    d.delay = arr(nw.delay, np.uint8)
    d.is_inh = arr(nw.is_inh, np.uint8)
    d.region = arr(nw.region, np.int32)
    d.ptype = arr(nw.ptype, np.uint16)
    ptypes = (Ptype * d.n_ptypes)()
    for p in range(d.n_ptypes):
        r = pt[p]
        ptypes[p] = Ptype(*[float(x) for x in r[:7]], (ctypes.c_float * 4)(*[float(x) for x in r[7:11]]))
    keep.append(ptypes)
    d.ptypes = ctypes.cast(ptypes, ctypes.c_void_p)
    d.V0 = arr(nw.V0, np.float32)
    for u in range(4):
        d.E[u] = float(nw.E[u])
        d.tau_ms[u] = float(nw.tau_ms[u])
    d.dt_ms = float(nw.dt_ms)
    d.bg_w = float(nw.bg_w)
    d.bg_lambda = float(nw.bg_lambda)
    d.seed = int(nw.seed)
    d.wtype = {"f32": W_F32, "bf16": W_BF16}[wtype]
    d.record_steps = int(record_steps)
    d.gather_bundle_syn = int(bundle_syn)
    d.gather_unroll = int(unroll)
    d.gather_fuse = int(fuse)
    d.gather_events = int(events)
    return d, keep


def pack_bits(raster: np.ndarray, words: int) -> np.ndarray:
    """[T, n] 0/1 -> [T, words] uint32 with neuron i at bit (i & 31) of word i >> 5."""
    T, n = raster.shape
    padded = np.zeros((T, words * 32), dtype=np.uint8)
    padded[:, :n] = raster
    b = np.packbits(padded, axis=-1, bitorder="little")          # [T, words * 4] bytes
    return np.ascontiguousarray(b).view("<u4").reshape(T, words)


def unpack_bits(bits: np.ndarray, n: int) -> np.ndarray:
    T, words = bits.shape
    by = np.ascontiguousarray(bits, dtype="<u4").view(np.uint8).reshape(T, words * 4)
    u = np.unpackbits(by, axis=-1, bitorder="little")
    return np.ascontiguousarray(u[:, :n])
