"""Python surface of libspiir: banks, tapes, batches and an autograd Function.

PyTorch provides device memory and the current HIP stream; every computation
is a call into the library (see include/spiir.h for the operations).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import BankInfo, call, default_opts, load


def _stream_ptr(stream=None) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _require_cuda(t: torch.Tensor, dtype, name: str):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError("%s must be a contiguous %s CUDA tensor" % (name, dtype))


def _c128(v) -> np.ndarray:
    arr = np.ascontiguousarray(np.asarray(v, dtype=np.complex128))
    return arr


class SpiirBank:
    """A device-resident SPIIR template bank with streaming state.

    offsets: int64 [T+1]; a, b: complex [F]; d: int [F]. Options as in
    spiir_bank_opts (chunk_len, filters_per_lane, max_delay, precision,
    device, max_block, waves_per_group, autotune).
    """

    def __init__(self, offsets, a, b, d, **opts):
        lib = load()
        self._off = np.ascontiguousarray(offsets, dtype=np.int64)
        self._a = _c128(a)
        self._b = _c128(b)
        self._d = np.ascontiguousarray(d, dtype=np.int32)
        o = default_opts()
        for k, v in opts.items():
            if not hasattr(o, k):
                raise TypeError("unknown bank option %r" % k)
            setattr(o, k, int(v))
        h = ctypes.c_void_p()
        call("spiir_bank_create", ctypes.byref(h), len(self._off) - 1,
             self._off.ctypes.data_as(ctypes.c_void_p), self._a.ctypes.data_as(ctypes.c_void_p),
             self._b.ctypes.data_as(ctypes.c_void_p), self._d.ctypes.data_as(ctypes.c_void_p),
             ctypes.byref(o))
        self._h = h
        self._lib = lib
        self.info = self.get_info()

    @classmethod
    def from_bank(cls, bank, **opts):
        """From a workloads.Bank (offsets, a, b, d, dmax)."""
        opts.setdefault("max_delay", int(bank.dmax))
        return cls(bank.offsets, bank.a, bank.b, bank.d, **opts)

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            call("spiir_bank_destroy", self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    # -- facts --------------------------------------------------------------
    def get_info(self) -> dict:
        info = BankInfo()
        call("spiir_bank_get_info", self._h, ctypes.byref(info))
        return info.as_dict()

    @property
    def n_templates(self) -> int:
        return self.info["n_templates"]

    @property
    def n_filters(self) -> int:
        return self.info["n_filters"]

    # -- state --------------------------------------------------------------
    def reset(self, stream=None):
        call("spiir_bank_reset", self._h, _stream_ptr(stream))

    def set_coeffs(self, a, b):
        self._a = _c128(a)
        self._b = _c128(b)
        call("spiir_bank_set_coeffs", self._h, self._a.ctypes.data_as(ctypes.c_void_p),
             self._b.ctypes.data_as(ctypes.c_void_p))

    def set_coeffs_dev(self, a: torch.Tensor, b: torch.Tensor, stream=None):
        """Replaces a, b from complex128 CUDA tensors [F] (caller order), on the
        stream; the values are not checked (keep |a| < 1)."""
        for t, name in ((a, "a"), (b, "b")):
            _require_cuda(t, torch.complex128, name)
            if t.numel() != self.n_filters:
                raise ValueError("%s must hold %d coefficients" % (name, self.n_filters))
        call("spiir_bank_set_coeffs_dev", self._h, _ptr(a), _ptr(b), _stream_ptr(stream))

    def get_state(self) -> bytes:
        n = ctypes.c_size_t()
        call("spiir_bank_state_size", self._h, ctypes.byref(n))
        buf = ctypes.create_string_buffer(n.value)
        call("spiir_bank_get_state", self._h, buf, n.value)
        return buf.raw

    def set_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        call("spiir_bank_set_state", self._h, buf, len(blob))

    # -- kernel timing ------------------------------------------------------
    def time_kernels(self, enable: bool = True):
        call("spiir_bank_time_kernels", self._h, 1 if enable else 0)

    def kernel_time(self):
        """(total ms, launches) of the forward kernels since the last read."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        call("spiir_bank_kernel_time", self._h, ctypes.byref(ms), ctypes.byref(n))
        return ms.value, n.value

    # -- forward ------------------------------------------------------------
    def filter_block(self, x: torch.Tensor, snr: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Next len(x) samples -> SNR of every template, float32 [T, n]. snr may
        be a column slice of a longer row-major array (rows of stride ld >= n)."""
        _require_cuda(x, torch.float32, "x")
        n = x.numel()
        if snr is None:
            snr = torch.empty((self.n_templates, n), dtype=torch.float32, device=x.device)
        if not (snr.is_cuda and snr.dtype == torch.float32 and snr.dim() == 2 and snr.stride(1) == 1
                and snr.shape[0] == self.n_templates and snr.shape[1] == n and snr.stride(0) >= n):
            raise ValueError("snr must be a float32 CUDA array [T, n] with unit column stride")
        call("spiir_filter_block", self._h, _ptr(x), n, _ptr(snr), snr.stride(0), _stream_ptr(stream))
        return snr

    def filter_block_z(self, x: torch.Tensor, z: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Next len(x) samples -> complex template sums, complex64 [T, n]."""
        _require_cuda(x, torch.float32, "x")
        n = x.numel()
        if z is None:
            z = torch.empty((self.n_templates, n), dtype=torch.complex64, device=x.device)
        _require_cuda(z, torch.complex64, "z")
        call("spiir_filter_block_z", self._h, _ptr(x), n, _ptr(z), z.shape[-1], _stream_ptr(stream))
        return z

    def trigger_max(self, x: torch.Tensor, out=None, stream=None):
        """Next len(x) samples -> (max SNR over templates float32 [n], argmax int32 [n])."""
        _require_cuda(x, torch.float32, "x")
        n = x.numel()
        if out is None:
            out = (torch.empty(n, dtype=torch.float32, device=x.device),
                   torch.empty(n, dtype=torch.int32, device=x.device))
        mx, am = out
        call("spiir_trigger_max", self._h, _ptr(x), n, _ptr(mx), _ptr(am), _stream_ptr(stream))
        return mx, am

    def trigger_max_noalloc(self, x: torch.Tensor, out, stream=None):
        """trigger_max whose working memory is the library's fixed per-device
        array (no device allocation in the call); out = (max float32 [n],
        argmax int32 [n]) is required."""
        _require_cuda(x, torch.float32, "x")
        n = x.numel()
        mx, am = out
        _require_cuda(mx, torch.float32, "max")
        _require_cuda(am, torch.int32, "argmax")
        if mx.numel() < n or am.numel() < n:
            raise ValueError("outputs hold fewer than len(x) samples")
        call("spiir_trigger_max_noalloc", self._h, _ptr(x), n, _ptr(mx), _ptr(am), _stream_ptr(stream))
        return mx, am

    def trigger_max_per_template(self, x: torch.Tensor, out=None, snr_scratch=None, stream=None):
        """Same outputs as trigger_max via one launch per template plus a max pass."""
        _require_cuda(x, torch.float32, "x")
        n = x.numel()
        if out is None:
            out = (torch.empty(n, dtype=torch.float32, device=x.device),
                   torch.empty(n, dtype=torch.int32, device=x.device))
        if snr_scratch is None:
            snr_scratch = torch.empty((self.n_templates, n), dtype=torch.float32, device=x.device)
        mx, am = out
        call("spiir_trigger_max_per_template", self._h, _ptr(x), n, _ptr(mx), _ptr(am),
             _ptr(snr_scratch), _stream_ptr(stream))
        return mx, am

    def forward_z(self, x: torch.Tensor, want_tape: bool = False, stream=None):
        """One-shot forward from a cold start: z complex64 [T, n] (and a Tape)."""
        _require_cuda(x, torch.float32, "x")
        n = x.numel()
        z = torch.empty((self.n_templates, n), dtype=torch.complex64, device=x.device)
        tp = ctypes.c_void_p()
        call("spiir_forward_z", self._h, _ptr(x), n, _ptr(z),
             ctypes.byref(tp) if want_tape else None, _stream_ptr(stream))
        return (z, Tape(tp, self)) if want_tape else z

    def backward(self, tape: "Tape", grad_z: torch.Tensor, stream=None):
        """Adjoint: grad_z complex64 [T, n] -> (grad_a, grad_b) complex64 [F]."""
        _require_cuda(grad_z, torch.complex64, "grad_z")
        F = self.n_filters
        ga = torch.empty(F, dtype=torch.complex64, device=grad_z.device)
        gb = torch.empty(F, dtype=torch.complex64, device=grad_z.device)
        call("spiir_backward", self._h, tape.handle, _ptr(grad_z), _ptr(ga), _ptr(gb), _stream_ptr(stream))
        return ga, gb


class Tape:
    """Chunk-start carries kept by forward_z for the adjoint."""

    def __init__(self, h, bank):
        self._h = h
        self._bank = bank

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            torch.cuda.synchronize()
            call("spiir_tape_destroy", self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SpiirBatch:
    """Several banks advanced one block per step by one graph replay."""

    def __init__(self, banks, xs, block_len: int = 4096, stream=None):
        self.banks = list(banks)
        self.xs = list(xs)
        for x in self.xs:
            _require_cuda(x, torch.float32, "x")
        dev = self.xs[0].device
        self.max = [torch.empty(x.numel(), dtype=torch.float32, device=dev) for x in self.xs]
        self.argmax = [torch.empty(x.numel(), dtype=torch.int32, device=dev) for x in self.xs]
        ns = len(self.banks)
        VP = ctypes.c_void_p * ns
        self._bh = VP(*[b.handle.value for b in self.banks])
        self._xh = VP(*[x.data_ptr() for x in self.xs])
        self._mh = VP(*[m.data_ptr() for m in self.max])
        self._ah = VP(*[a.data_ptr() for a in self.argmax])
        self._len = (ctypes.c_int64 * ns)(*[x.numel() for x in self.xs])
        h = ctypes.c_void_p()
        call("spiir_batch_create", ctypes.byref(h), ns, self._bh, self._xh, self._len, self._mh,
             self._ah, int(block_len), _stream_ptr(stream))
        self._h = h
        self.block_len = int(block_len)

    def step(self, stream=None):
        call("spiir_batch_step", self._h, _stream_ptr(stream))

    def set_time_split(self, mode: int):
        """0 = automatic graph choice, 1 = plain graph only, 2 = time-split graph only."""
        call("spiir_batch_set_time_split", self._h, int(mode))

    def steps_total(self) -> int:
        v = ctypes.c_int64()
        call("spiir_batch_steps_total", self._h, ctypes.byref(v))
        return int(v.value)

    def reset(self, stream=None):
        call("spiir_batch_reset", self._h, _stream_ptr(stream))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            call("spiir_batch_destroy", self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(banks, block_len: int = 4096, max_delay: int = 0, device: int = -1):
    """Times (chunk_len, filters_per_lane) candidates on workloads.Bank-like
    objects run as one batch; returns (chunk_len, filters_per_lane, table[4][4] ns)."""
    n = len(banks)
    offs = [np.ascontiguousarray(b.offsets, dtype=np.int64) for b in banks]
    aas = [_c128(b.a) for b in banks]
    bbs = [_c128(b.b) for b in banks]
    dds = [np.ascontiguousarray(b.d, dtype=np.int32) for b in banks]
    VP = ctypes.c_void_p * n
    T = (ctypes.c_int32 * n)(*[len(o) - 1 for o in offs])
    L = ctypes.c_int32()
    F = ctypes.c_int32()
    table = (ctypes.c_float * 16)()
    call("spiir_autotune", n, T, VP(*[o.ctypes.data for o in offs]), VP(*[a.ctypes.data for a in aas]),
         VP(*[b.ctypes.data for b in bbs]), VP(*[d.ctypes.data for d in dds]), int(max_delay),
         int(block_len), int(device), ctypes.byref(L), ctypes.byref(F), table)
    return int(L.value), int(F.value), np.array(list(table), dtype=np.float64).reshape(4, 4)


def batch_banks(banks, chunk_len: int, filters_per_lane: int, device: int = 0, **opts):
    """SpiirBanks for several workloads.Bank objects with one common layout
    (filters per lane, chunk length and workgroup size), as a batch needs.
    The workgroup size spreads all banks' rows over the device's CUs."""
    rows = lambda k: -(-int(k) // (16 * filters_per_lane))  # noqa: E731
    total = sum(rows(k) for b in banks for k in np.diff(b.offsets))
    max_nr = max(rows(k) for b in banks for k in np.diff(b.offsets))
    n_cu = torch.cuda.get_device_properties(device).multi_processor_count
    waves = -(-total // 4)
    wpg = min(8, max(-(-waves // n_cu), -(-max_nr // 4)))
    return [SpiirBank.from_bank(b, chunk_len=chunk_len, filters_per_lane=filters_per_lane,
                                waves_per_group=wpg, device=device, **opts) for b in banks]


class SpiirFn(torch.autograd.Function):
    """z = bank(x) from a cold start, differentiable in the coefficients.

    forward(ctx, a, b, bank, x): a, b complex128 tensors [F] (set into the
    bank: from the device when they live on the bank's GPU, else through the
    host), x float32 CUDA [n]; returns z complex64 CUDA [T, n]. backward runs
    the library's reverse-time adjoint and returns complex128 gradients on
    a's device in PyTorch's convention (dL/dRe + i dL/dIm).
    """

    @staticmethod
    def forward(ctx, a, b, bank: SpiirBank, x: torch.Tensor):
        if a.is_cuda and b.is_cuda:
            bank.set_coeffs_dev(a.detach().contiguous(), b.detach().contiguous())
        else:
            bank.set_coeffs(a.detach().cpu().numpy(), b.detach().cpu().numpy())
        z, tape = bank.forward_z(x, want_tape=True)
        ctx.bank = bank
        ctx.tape = tape
        ctx.a_dev = a.device
        return z

    @staticmethod
    def backward(ctx, grad_z):
        gz = grad_z.to(torch.complex64).contiguous()
        ga, gb = ctx.bank.backward(ctx.tape, gz)
        ctx.tape.close()
        return (ga.to(torch.complex128).to(ctx.a_dev), gb.to(torch.complex128).to(ctx.a_dev),
                None, None)


def _cuda_device(device=None) -> torch.device:
    """torch.device with an explicit index (the current device when none is given)."""
    dev = torch.device("cuda") if device is None else torch.device(device)
    if dev.type != "cuda":
        raise ValueError("a CUDA device is required (got %s)" % dev)
    return torch.device("cuda", torch.cuda.current_device() if dev.index is None else dev.index)


class SpiirMultiRate:
    """Multi-rate bank (spiir_multirate_*): `levels` is a list of
    workloads.Bank-like objects, level r running at 1 / 2^r of the input
    rate, all with the same templates (a template may have no filters at a
    level); h and g are the decimation and interpolation taps."""

    def __init__(self, levels, h, g, **opts):
        o = default_opts()
        for k, v in opts.items():
            setattr(o, k, v)
        self.n_levels = len(levels)
        T = levels[0].n_templates
        self._keep = []
        offs, aas, bbs, dds = [], [], [], []
        for lv in levels:
            off = np.ascontiguousarray(lv.offsets, dtype=np.int64)
            a, b = _c128(lv.a), _c128(lv.b)
            d = np.ascontiguousarray(lv.d, dtype=np.int32)
            self._keep += [off, a, b, d]
            offs.append(off.ctypes.data)
            empty = int(off[-1]) == 0
            aas.append(None if empty else a.ctypes.data)
            bbs.append(None if empty else b.ctypes.data)
            dds.append(None if empty else d.ctypes.data)
        VP = ctypes.c_void_p * self.n_levels
        hh = np.ascontiguousarray(h, dtype=np.float64)
        gg = np.ascontiguousarray(g, dtype=np.float64)
        self._h = ctypes.c_void_p()
        call("spiir_multirate_create", ctypes.byref(self._h), self.n_levels, T, VP(*offs), VP(*aas), VP(*bbs),
             VP(*dds), hh.ctypes.data_as(ctypes.c_void_p), len(hh), gg.ctypes.data_as(ctypes.c_void_p), len(gg),
             ctypes.byref(o))
        self.n_templates = T
        self.block_multiple = 1 << (self.n_levels - 1)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().spiir_multirate_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def reset(self, stream=None):
        call("spiir_multirate_reset", self._h, _stream_ptr(stream))

    def filter_block_z(self, x: torch.Tensor, z: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Full-rate template sums, complex64 [T, n]."""
        _require_cuda(x, torch.float32, "x")
        n = x.numel()
        if z is None:
            z = torch.empty((self.n_templates, n), dtype=torch.complex64, device=x.device)
        call("spiir_multirate_filter_block_z", self._h, _ptr(x), n, _ptr(z), z.shape[-1], _stream_ptr(stream))
        return z

    def trigger_max(self, x: torch.Tensor, out=None, stream=None):
        _require_cuda(x, torch.float32, "x")
        n = x.numel()
        if out is None:
            out = (torch.empty(n, dtype=torch.float32, device=x.device),
                   torch.empty(n, dtype=torch.int32, device=x.device))
        mx, am = out
        call("spiir_multirate_trigger_max", self._h, _ptr(x), n, _ptr(mx), _ptr(am), _stream_ptr(stream))
        return mx, am

    def set_graph(self, enable: bool):
        """Graph replay of trigger pieces of exactly max_block samples (on by default)."""
        call("spiir_multirate_set_graph", self._h, 1 if enable else 0)

    def level_info(self, level: int):
        """Layout facts of the bank running `level`, or None when it holds no filters."""
        bh = ctypes.c_void_p()
        call("spiir_multirate_level_bank", self._h, int(level), ctypes.byref(bh))
        if not bh.value:
            return None
        info = BankInfo()
        call("spiir_bank_get_info", bh, ctypes.byref(info))
        return info.as_dict()

    def level_bank_handle(self, level: int):
        bh = ctypes.c_void_p()
        call("spiir_multirate_level_bank", self._h, int(level), ctypes.byref(bh))
        return bh if bh.value else None

    def time_kernels(self, enable: bool = True):
        """Forward-kernel timing of every level's bank (spiir_bank_time_kernels)."""
        for r in range(self.n_levels):
            bh = self.level_bank_handle(r)
            if bh is not None:
                call("spiir_bank_time_kernels", bh, 1 if enable else 0)

    def kernel_time(self):
        """{level: (total ms, launches)} of the level banks' forward kernels since the last read."""
        out = {}
        for r in range(self.n_levels):
            bh = self.level_bank_handle(r)
            if bh is not None:
                ms, n = ctypes.c_double(), ctypes.c_int64()
                call("spiir_bank_kernel_time", bh, ctypes.byref(ms), ctypes.byref(n))
                out[r] = (ms.value, n.value)
        return out


class Whitener:
    """Whitening front end (spiir_whitener_*): Welch PSD of a training
    stretch and frame-wise whitening with overlap-add; the output is the
    whitened stream delayed by frame_len / 2 samples."""

    def __init__(self, frame_len: int = 4096, max_block: int = 0, device: int = -1):
        self._h = ctypes.c_void_p()
        call("spiir_whitener_create", ctypes.byref(self._h), int(frame_len), int(max_block), int(device))
        self.frame_len = int(frame_len)
        self.hop = self.frame_len // 2

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().spiir_whitener_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def estimate_psd(self, train: torch.Tensor, stream=None):
        _require_cuda(train, torch.float32, "train")
        call("spiir_whitener_estimate_psd", self._h, _ptr(train), train.numel(), _stream_ptr(stream))

    def set_psd(self, psd):
        p = np.ascontiguousarray(psd, dtype=np.float64)
        if p.shape != (self.hop + 1,):
            raise ValueError("psd must have frame_len / 2 + 1 values")
        call("spiir_whitener_set_psd", self._h, p.ctypes.data_as(ctypes.c_void_p))

    def psd(self) -> np.ndarray:
        p = np.zeros(self.hop + 1, np.float64)
        call("spiir_whitener_get_psd", self._h, p.ctypes.data_as(ctypes.c_void_p))
        return p

    def process(self, x: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        _require_cuda(x, torch.float32, "x")
        if out is None:
            out = torch.empty_like(x)
        _require_cuda(out, torch.float32, "out")
        call("spiir_whitener_process", self._h, _ptr(x), x.numel(), _ptr(out), _stream_ptr(stream))
        return out

    def reset(self, stream=None):
        call("spiir_whitener_reset", self._h, _stream_ptr(stream))


class TriggerClusterer:
    """Trigger clustering of max/argmax series of up to max_n samples with a
    preallocated device workspace and outputs for `capacity` triggers
    (spiir_cluster_triggers). run() only enqueues work; result() waits for it."""

    def __init__(self, max_n: int, capacity: int, device=None):
        dev = _cuda_device(device)
        nb = ctypes.c_size_t()
        call("spiir_cluster_workspace_size", int(max_n), ctypes.byref(nb))
        self.max_n, self.capacity, self.device = int(max_n), int(capacity), dev
        self.workspace = torch.empty(max(1, nb.value), dtype=torch.uint8, device=dev)
        self.index = torch.empty(max(1, self.capacity), dtype=torch.int64, device=dev)
        self.template = torch.empty(max(1, self.capacity), dtype=torch.int32, device=dev)
        self.snr = torch.empty(max(1, self.capacity), dtype=torch.float32, device=dev)
        self.count = torch.zeros(1, dtype=torch.int64, device=dev)

    def run(self, mx: torch.Tensor, am: torch.Tensor, threshold: float, window: int, stream=None):
        _require_cuda(mx, torch.float32, "max")
        _require_cuda(am, torch.int32, "argmax")
        n = mx.numel()
        if am.numel() != n:
            raise ValueError("max and argmax differ in length")
        if n > self.max_n:
            raise ValueError("series of %d samples exceeds max_n = %d" % (n, self.max_n))
        if mx.device != self.device or am.device != self.device:
            raise ValueError("series are not on %s" % self.device)
        call("spiir_cluster_triggers", _ptr(mx), _ptr(am), n, float(threshold), int(window),
             _ptr(self.workspace), self.workspace.numel(), _ptr(self.index), _ptr(self.template),
             _ptr(self.snr), self.capacity, _ptr(self.count), self.device.index, _stream_ptr(stream))

    def result(self):
        """(index, template, snr, total): the first min(total, capacity)
        triggers and the total count."""
        total = int(self.count.item())
        k = min(total, self.capacity)
        return self.index[:k], self.template[:k], self.snr[:k], total


class TriggerStream:
    """Streaming trigger clustering (spiir_trigger_stream_*): push each block's
    max / argmax; every push returns the triggers that became final (W samples
    of latency), flush() returns the rest at the end of the stream."""

    def __init__(self, threshold: float, window: int, max_block: int, capacity: int | None = None,
                 device=None):
        dev = _cuda_device(device)
        self._h = ctypes.c_void_p()
        call("spiir_trigger_stream_create", ctypes.byref(self._h), float(threshold), int(window), int(max_block),
             dev.index)
        self.device = dev
        self.capacity = int(capacity) if capacity is not None else (max_block + window) // (window + 1) + 2
        self.index = torch.empty(max(1, self.capacity), dtype=torch.int64, device=dev)
        self.template = torch.empty(max(1, self.capacity), dtype=torch.int32, device=dev)
        self.snr = torch.empty(max(1, self.capacity), dtype=torch.float32, device=dev)
        self.count = torch.zeros(1, dtype=torch.int64, device=dev)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().spiir_trigger_stream_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _result(self):
        total = int(self.count.item())
        k = min(total, self.capacity)
        return self.index[:k].clone(), self.template[:k].clone(), self.snr[:k].clone(), total

    def push(self, mx: torch.Tensor, am: torch.Tensor, stream=None):
        """(index, template, snr, total) of the triggers that became final."""
        _require_cuda(mx, torch.float32, "max")
        _require_cuda(am, torch.int32, "argmax")
        if mx.numel() != am.numel():
            raise ValueError("max and argmax differ in length")
        call("spiir_trigger_stream_push", self._h, _ptr(mx), _ptr(am), mx.numel(), _ptr(self.index),
             _ptr(self.template), _ptr(self.snr), self.capacity, _ptr(self.count), _stream_ptr(stream))
        return self._result()

    def push_into(self, mx: torch.Tensor, am: torch.Tensor, index: torch.Tensor, template: torch.Tensor,
                  snr: torch.Tensor, count: torch.Tensor, stream=None):
        """Enqueues a push writing into caller tensors (no host synchronisation):
        up to index.numel() triggers, their total to count[0]."""
        _require_cuda(mx, torch.float32, "max")
        _require_cuda(am, torch.int32, "argmax")
        cap = index.numel()
        if template.numel() < cap or snr.numel() < cap or count.numel() < 1:
            raise ValueError("output tensors too small")
        call("spiir_trigger_stream_push", self._h, _ptr(mx), _ptr(am), mx.numel(), _ptr(index), _ptr(template),
             _ptr(snr), cap, _ptr(count), _stream_ptr(stream))

    def flush_into(self, index: torch.Tensor, template: torch.Tensor, snr: torch.Tensor, count: torch.Tensor,
                   stream=None):
        """Enqueues the end-of-stream flush writing into caller tensors."""
        cap = index.numel()
        if template.numel() < cap or snr.numel() < cap or count.numel() < 1:
            raise ValueError("output tensors too small")
        call("spiir_trigger_stream_flush", self._h, _ptr(index), _ptr(template), _ptr(snr), cap, _ptr(count),
             _stream_ptr(stream))

    def flush(self, stream=None):
        call("spiir_trigger_stream_flush", self._h, _ptr(self.index), _ptr(self.template), _ptr(self.snr),
             self.capacity, _ptr(self.count), _stream_ptr(stream))
        return self._result()

    def reset(self, stream=None):
        call("spiir_trigger_stream_reset", self._h, _stream_ptr(stream))


def cluster_triggers(mx: torch.Tensor, am: torch.Tensor, threshold: float, window: int,
                     capacity: int | None = None, stream=None):
    """One-shot clustering of a max/argmax series; the default capacity holds
    every possible trigger (they are more than `window` samples apart).
    Returns (index int64, template int32, snr float32, total)."""
    n = mx.numel()
    cap = n // (int(window) + 1) + 1 if capacity is None else int(capacity)
    c = TriggerClusterer(n, cap, device=mx.device)
    c.run(mx, am, threshold, window, stream=stream)
    return c.result()


def version() -> str:
    return load().spiir_version().decode()


__all__ = ["SpiirBank", "SpiirBatch", "SpiirFn", "SpiirMultiRate", "Tape", "TriggerClusterer", "TriggerStream", "Whitener", "autotune",
           "batch_banks",
           "cluster_triggers", "version", "_lib"]
