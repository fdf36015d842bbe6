"""Period-window proposal network: binding of the ``cetra_net_*`` calls.

The network is an addition to the paper's method: it scores log-spaced
period windows from the linear search's single-event statistics (Sec. 2.2),
and the periodic search (Sec. 2.3) then folds only the periods of the K
best-scored windows.  Every forward, backward and optimiser stage runs in the
library's HIP kernels; this module owns the device buffers and sequences the
calls.

Parameters live in one flat FP32 device buffer (masters), with gradients and
Adam moments in buffers of the same layout, so one kernel clears the
gradients and one applies Adam.  Conv weights are stored as [64][k32]
(k = tap * cin + ci, zero padding columns) and packed to bfloat16 for the
MFMA convolutions after every update.
"""

from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np

from . import _abi
from . import _ptr, _stream

WIDTH = 64
N_LAYERS = 5
C_IN = 16
TAPS = 9


def _k32(cin: int) -> int:
    return (TAPS * cin + 31) // 32 * 32


def _lib():
    return _abi.load()


@dataclass
class Windows:
    """Log-spaced period windows over [p_lo, p_hi] days on an axis of bins of
    bin_days: window w covers periods [edges[w], edges[w+1]); q[w] is its
    position (w + 1/2) / n in [0, 1]."""

    q: np.ndarray
    edges: np.ndarray
    bin_days: float

    @classmethod
    def log_spaced(cls, n: int, p_lo: float, p_hi: float, bin_days: float) -> "Windows":
        if not (n >= 1 and 0 < p_lo < p_hi and bin_days > 0):
            raise ValueError("windows: need n >= 1, 0 < p_lo < p_hi, bin_days > 0")
        edges = p_lo * np.power(p_hi / p_lo, np.arange(n + 1, dtype=np.float64) / n)
        q = ((np.arange(n) + 0.5) / n).astype(np.float32)
        return cls(q, edges, float(bin_days))

    @property
    def n(self) -> int:
        return int(self.q.shape[0])

    def device(self):
        import torch
        if not hasattr(self, "_dev"):
            self._dev = dict(q=torch.as_tensor(self.q, device="cuda"), edges=torch.as_tensor(self.edges, device="cuda"))
        return self._dev

    def trials(self, n_trial: int) -> np.ndarray:
        """Trial periods in bins of every window [W][n_trial]: the centres of
        n_trial equal log-steps of [edges[w], edges[w+1])."""
        frac = (np.arange(n_trial) + 0.5) / n_trial
        lo, hi = self.edges[:-1, None], self.edges[1:, None]
        return lo * (hi / lo) ** frac[None, :] / self.bin_days

    def trials_device(self, n_trial: int):
        import torch
        key = f"_trials{n_trial}"
        if not hasattr(self, key):
            setattr(self, key, torch.as_tensor(np.ascontiguousarray(self.trials(n_trial)), device="cuda"))
        return getattr(self, key)

    def labels(self, periods) -> np.ndarray:
        """One-hot window index of each true period (all zero when a period
        lies outside the windows)."""
        periods = np.atleast_1d(np.asarray(periods, dtype=np.float64))
        y = np.zeros((periods.shape[0], self.n), dtype=np.float32)
        w = np.searchsorted(self.edges, periods, side="right") - 1
        ok = (w >= 0) & (w < self.n)
        y[np.nonzero(ok)[0], w[ok]] = 1.0
        return y


class ProposalNet:
    """Five 9-tap convolutions of 64 channels (ReLU), a linear 1x1
    projection to E event channels, fold pooling -- the coarse fold of each
    event channel at S trial periods per window, keeping the best phase
    score -- and a shared MLP head (hidden width H) giving one logit per
    window."""

    def __init__(self, n_event: int = 8, hidden: int = 64, seed: int = 0, n_trial: int = 4):
        import torch
        self.E, self.H = int(n_event), int(hidden)
        if not (1 <= self.E <= 16 and 1 <= self.H <= 128 and 1 <= n_trial <= 32):
            raise ValueError("proposal net: need 1 <= n_event <= 16, 1 <= hidden <= 128, 1 <= n_trial <= 32")
        self.S = int(n_trial)
        self.signed_input = False  # input features: |SNR| (False) or signed SNR (True)
        self.nf = self.E + 1
        shapes = []
        cin = C_IN
        for l in range(N_LAYERS):
            shapes += [(f"W{l}", (WIDTH, _k32(cin))), (f"b{l}", (WIDTH,))]
            cin = WIDTH
        shapes += [("P", (self.E, WIDTH)), ("p", (self.E,)), ("U", (self.H, self.nf)), ("u", (self.H,)),
                   ("v", (self.H,)), ("v0", (1,))]
        self.offsets, off = {}, 0
        for name, shp in shapes:
            n = int(np.prod(shp))
            off = (off + 63) // 64 * 64  # 256-byte aligned views
            self.offsets[name] = (off, shp)
            off += n
        self.n_flat = off
        dev = "cuda"
        self.flat = torch.zeros(off, dtype=torch.float32, device=dev)
        self.grad = torch.zeros_like(self.flat)
        self.m = torch.zeros_like(self.flat)
        self.v = torch.zeros_like(self.flat)
        self.step_count = 0
        self.packed = [torch.zeros((WIDTH, _k32(C_IN if l == 0 else WIDTH)), dtype=torch.bfloat16, device=dev)
                       for l in range(N_LAYERS)]
        self.init(seed)
        self._bufs = {}

    # ------------------------------------------------------------ parameters
    def view(self, name, which=None):
        off, shp = self.offsets[name]
        buf = self.flat if which is None else which
        return buf[off:off + int(np.prod(shp))].view(*shp)

    def init(self, seed: int) -> None:
        """He-style initialisation (normal, std sqrt(2 / fan_in)) on the host
        with a seeded generator; padding columns zero."""
        rng = np.random.default_rng(seed)
        arrays = {}
        cin = C_IN
        for l in range(N_LAYERS):
            w = np.zeros((WIDTH, _k32(cin)))
            w[:, :TAPS * cin] = rng.normal(0, math.sqrt(2.0 / (TAPS * cin)), (WIDTH, TAPS * cin))
            arrays[f"W{l}"] = w
            arrays[f"b{l}"] = np.zeros(WIDTH)
            cin = WIDTH
        arrays["P"] = rng.normal(0, math.sqrt(2.0 / WIDTH), (self.E, WIDTH))
        arrays["p"] = np.full(self.E, 0.01)
        arrays["U"] = rng.normal(0, math.sqrt(2.0 / self.nf), (self.H, self.nf))
        arrays["u"] = np.zeros(self.H)
        arrays["v"] = rng.normal(0, math.sqrt(1.0 / self.H), self.H)
        arrays["v0"] = np.array([-2.0])
        self._load(arrays)

    def _load(self, arrays: dict) -> None:
        import torch
        for name, a in arrays.items():
            self.view(name).copy_(torch.as_tensor(np.asarray(a, dtype=np.float32)))
        self.pack()

    def load_arrays(self, arrays: dict) -> None:
        """Load parameters given with conv weights as [64][cin][9] (output,
        input channel, tap) -- the cross-correlation's natural layout."""
        conv = {}
        for name, a in arrays.items():
            if name.startswith("W"):
                a = np.asarray(a)
                o, cin, taps = a.shape
                w = np.zeros((o, _k32(cin)))
                w[:, :taps * cin] = np.transpose(a, (0, 2, 1)).reshape(o, taps * cin)
                conv[name] = w
            else:
                conv[name] = np.asarray(a).reshape(self.offsets[name][1])
        self._load(conv)

    def grad_arrays(self) -> dict:
        """Gradients as host arrays, conv weights as [64][cin][9]."""
        out = {}
        cin = C_IN
        for name in self.offsets:
            g = self.view(name, self.grad).double().cpu().numpy()
            if name.startswith("W"):
                l = int(name[1:])
                cin = C_IN if l == 0 else WIDTH
                g = g[:, :TAPS * cin].reshape(WIDTH, TAPS, cin).transpose(0, 2, 1)
            out[name] = g
        return out

    def pack(self, stream=None) -> None:
        lib, s = _lib(), _stream(stream)
        for l in range(N_LAYERS):
            cin = C_IN if l == 0 else WIDTH
            _abi.check(lib.cetra_net_pack_conv_w(s, _ptr(self.view(f"W{l}")), cin, _k32(cin), _ptr(self.packed[l])))

    # --------------------------------------------------------------- buffers
    def _buffers(self, B: int, L: int, win: Windows):
        import torch
        key = (B, L, win.n)
        if key in self._bufs:
            return self._bufs[key]
        dev, f32, bf = "cuda", torch.float32, torch.bfloat16
        b = dict(
            h=[None] + [torch.empty((B, L, WIDTH), dtype=bf, device=dev) for _ in range(N_LAYERS)],
            e=torch.empty((B, L, self.E), dtype=f32, device=dev),
            f=torch.empty((B, win.n, self.nf), dtype=f32, device=dev),
            arg=torch.empty((B, win.n, self.E), dtype=torch.int32, device=dev),
            z=torch.empty((B, win.n), dtype=f32, device=dev),
            gz=torch.empty((B, win.n), dtype=f32, device=dev),
            gf=torch.empty((B, win.n, self.nf), dtype=f32, device=dev),
            ge=torch.empty((B, L, self.E), dtype=f32, device=dev),
            dh=[torch.empty((B, L, WIDTH), dtype=f32, device=dev) for _ in range(2)],
            g_scratch=torch.empty((B, L, WIDTH), dtype=bf, device=dev),
            wt_scratch=torch.empty((WIDTH * TAPS * WIDTH,), dtype=bf, device=dev),
            w_partial=torch.empty((max(bwd_partial_floats(C_IN, L, B), bwd_partial_floats(WIDTH, L, B)),),
                                  dtype=f32, device=dev),
            loss=torch.zeros(1, dtype=f32, device=dev),
        )
        self._bufs = {key: b}  # keep one shape's buffers
        return b

    # --------------------------------------------------------------- forward
    def forward(self, x, win: Windows, stream=None):
        """x: device bf16 [B][L][16] -> logits z [B][W] (a view of an internal
        buffer, overwritten by the next call)."""
        import torch
        if x.dtype != torch.bfloat16 or x.dim() != 3 or x.shape[2] != C_IN:
            raise ValueError("proposal forward: x must be bfloat16 [B][L][16]")
        B, L = int(x.shape[0]), int(x.shape[1])
        if L > 8192:
            raise ValueError("proposal forward: L must be <= 8192")
        lib, s = _lib(), _stream(stream)
        bufs = self._buffers(B, L, win)
        bufs["h"][0] = x.contiguous()
        dw = win.device()
        cin = C_IN
        for l in range(N_LAYERS):
            _abi.check(lib.cetra_conv1d_fwd(s, _ptr(bufs["h"][l]), cin, L, B, _ptr(self.packed[l]), _k32(cin),
                                            _ptr(self.view(f"b{l}")), _ptr(bufs["h"][l + 1])))
            cin = WIDTH
        _abi.check(lib.cetra_net_project_fwd(s, _ptr(bufs["h"][N_LAYERS]), B * L, _ptr(self.view("P")),
                                             _ptr(self.view("p")), self.E, _ptr(bufs["e"])))
        _abi.check(lib.cetra_net_foldpool_fwd(s, _ptr(bufs["e"]), B, L, self.E, _ptr(win.trials_device(self.S)),
                                              win.n, self.S, _ptr(dw["q"]), _ptr(bufs["f"]), _ptr(bufs["arg"])))
        _abi.check(lib.cetra_net_head_fwd(s, _ptr(bufs["f"]), B * win.n, self.nf, _ptr(self.view("U")),
                                          _ptr(self.view("u")), _ptr(self.view("v")), _ptr(self.view("v0")), self.H,
                                          _ptr(bufs["z"])))
        self._last = (B, L, win)
        return bufs["z"]

    # -------------------------------------------------------------- backward
    def backward(self, y, pos_weight: float = 1.0, stream=None, want_dx: bool = False):
        """Loss and parameter gradients (into self.grad, cleared first) for
        labels y [B][W] (device FP32 0/1) after forward().  Returns the loss
        as a device scalar tensor (and dL/dx [B][L][16] FP32 when asked)."""
        import torch
        B, L, win = self._last
        lib, s = _lib(), _stream(stream)
        bufs = self._bufs[(B, L, win.n)]
        self.grad.zero_()
        bufs["loss"].zero_()
        n_bw = B * win.n
        _abi.check(lib.cetra_net_bce(s, _ptr(bufs["z"]), _ptr(y), n_bw, float(pos_weight), _ptr(bufs["gz"]),
                                     _ptr(bufs["loss"])))
        _abi.check(lib.cetra_net_head_bwd(s, _ptr(bufs["f"]), n_bw, self.nf, _ptr(self.view("U")),
                                          _ptr(self.view("u")), _ptr(self.view("v")), self.H, _ptr(bufs["gz"]),
                                          _ptr(self.view("U", self.grad)), _ptr(self.view("u", self.grad)),
                                          _ptr(self.view("v", self.grad)), _ptr(self.view("v0", self.grad)),
                                          _ptr(bufs["gf"])))
        _abi.check(lib.cetra_net_foldpool_bwd(s, _ptr(bufs["gf"]), _ptr(bufs["arg"]), _ptr(win.trials_device(self.S)),
                                              B, L, self.E, win.n, self.S, _ptr(bufs["ge"])))
        dh_in, dh_out = bufs["dh"]
        _abi.check(lib.cetra_net_project_bwd(s, _ptr(bufs["h"][N_LAYERS]), _ptr(bufs["ge"]), B * L,
                                             _ptr(self.view("P")), self.E, _ptr(dh_in),
                                             _ptr(self.view("P", self.grad)), _ptr(self.view("p", self.grad))))
        dx = None
        for l in reversed(range(N_LAYERS)):
            cin = C_IN if l == 0 else WIDTH
            if l == 0:
                dx = torch.empty((B, L, C_IN), dtype=torch.float32, device="cuda") if want_dx else None
                out = dx
            else:
                out = dh_out
            _abi.check(lib.cetra_conv1d_bwd(s, _ptr(dh_in), _ptr(bufs["h"][l + 1]), _ptr(bufs["h"][l]), cin, L, B,
                                            _ptr(self.packed[l]), _k32(cin), _ptr(bufs["g_scratch"]),
                                            _ptr(bufs["wt_scratch"]), _ptr(bufs["w_partial"]),
                                            bufs["w_partial"].numel(), _ptr(out) if out is not None else None,
                                            _ptr(self.view(f"W{l}", self.grad)), _ptr(self.view(f"b{l}", self.grad))))
            dh_in, dh_out = dh_out, dh_in
        return (bufs["loss"], dx) if want_dx else bufs["loss"]

    def adam(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None):
        """One Adam step on every parameter, then repack the bf16 weights."""
        self.step_count += 1
        lib, s = _lib(), _stream(stream)
        _abi.check(lib.cetra_adam_step(s, _ptr(self.flat), _ptr(self.grad), _ptr(self.m), _ptr(self.v), self.n_flat,
                                       float(lr), float(beta1), float(beta2), float(eps), self.step_count))
        self.pack(stream)


# ------------------------------------------------------------------ helpers
def mfma_probe(a, b, stream=None):
    import torch
    c = torch.empty((16, 16), dtype=torch.float32, device="cuda")
    _abi.check(_lib().cetra_net_mfma_probe(_stream(stream), _ptr(a.contiguous()), _ptr(b.contiguous()), _ptr(c)))
    return c


def conv1d_fwd(x, w_packed, bias, stream=None):
    """x bf16 [B][L][cin], w_packed bf16 [64][k32], bias FP32 [64] -> y bf16."""
    import torch
    B, L, cin = (int(v) for v in x.shape)
    y = torch.empty((B, L, WIDTH), dtype=torch.bfloat16, device="cuda")
    _abi.check(_lib().cetra_conv1d_fwd(_stream(stream), _ptr(x), cin, L, B, _ptr(w_packed), int(w_packed.shape[1]),
                                       _ptr(bias), _ptr(y)))
    return y


def bwd_partial_floats(cin: int, L: int, B: int) -> int:
    """Floats of the weight-gradient partial-sum workspace (cetra_conv1d_bwd)."""
    n = int(_lib().cetra_conv1d_bwd_partial_floats(int(cin), int(L), int(B)))
    if n < 0:
        raise ValueError(f"conv1d_bwd: no workspace size for cin={cin}, L={L}, B={B}")
    return n


def conv1d_bwd(dy, y, x, w_packed, stream=None, partial: bool = True, dx_out: bool = True):
    """Returns dx [B][L][cin] FP32 (None with dx_out=False), dw [64][k32]
    FP32, db [64] FP32.  partial=False adds the weight gradient with
    atomics instead of the partial-sum workspace."""
    import torch
    B, L, cin = (int(v) for v in x.shape)
    k32 = int(w_packed.shape[1])
    dx = torch.empty((B, L, cin), dtype=torch.float32, device="cuda") if dx_out else None
    dw = torch.zeros((WIDTH, k32), dtype=torch.float32, device="cuda")
    db = torch.zeros(WIDTH, dtype=torch.float32, device="cuda")
    g = torch.empty((B, L, WIDTH), dtype=torch.bfloat16, device="cuda")
    wt = torch.empty(WIDTH * TAPS * cin, dtype=torch.bfloat16, device="cuda")
    part = torch.empty(bwd_partial_floats(cin, L, B), dtype=torch.float32, device="cuda") if partial else None
    _abi.check(_lib().cetra_conv1d_bwd(_stream(stream), _ptr(dy), _ptr(y), _ptr(x), cin, L, B, _ptr(w_packed), k32,
                                       _ptr(g), _ptr(wt), _ptr(part), part.numel() if partial else 0,
                                       _ptr(dx) if dx_out else None, _ptr(dw), _ptr(db)))
    return dx, dw, db


def downsample(fold, n_bins: int, out=None, signed: bool = False, stream=None):
    """fold-ready FP32 [J][I][2] -> bf16 [n_bins][J] single-event features:
    the bin's largest |SNR| (cetra_net_downsample), or with signed=True its
    largest signed SNR (cetra_net_downsample_signed)."""
    import torch
    J, I = int(fold.shape[0]), int(fold.shape[1])
    if out is None:
        out = torch.empty((n_bins, J), dtype=torch.bfloat16, device="cuda")
    fn = _lib().cetra_net_downsample_signed if signed else _lib().cetra_net_downsample
    _abi.check(fn(_stream(stream), _ptr(fold), J, I, int(n_bins), _ptr(out)))
    return out


def topk_windows(scores, k: int, stream=None):
    import torch
    B, W = (int(v) for v in scores.shape)
    out = torch.empty((B, k), dtype=torch.int32, device="cuda")
    _abi.check(_lib().cetra_topk_windows(_stream(stream), _ptr(scores.contiguous()), B, W, int(k), _ptr(out)))
    return out


def windows_to_periods(periods, win: Windows, sel, stream=None):
    """Device int64 indices of the periods (ascending, device FP64) inside
    the selected windows, and their count (device int64 [1])."""
    import torch
    K = int(periods.shape[0])
    subset = torch.empty(max(K, 1), dtype=torch.int64, device="cuda")
    n = torch.empty(1, dtype=torch.int64, device="cuda")
    sel = sel.reshape(-1).to(torch.int32).contiguous()
    _abi.check(_lib().cetra_windows_to_periods(_stream(stream), _ptr(periods), K, _ptr(win.device()["edges"]), win.n,
                                               _ptr(sel), int(sel.shape[0]), _ptr(subset), _ptr(n)))
    return subset, n


def foldpool_fwd(e, win: Windows, n_trial: int, stream=None):
    """Fold-pooling features f [B][W][E+1] and winners [B][W][E] of event
    series e [B][L][E] (device FP32) at the windows' trial periods."""
    import torch
    B, L, E = (int(v) for v in e.shape)
    f = torch.empty((B, win.n, E + 1), dtype=torch.float32, device="cuda")
    arg = torch.empty((B, win.n, E), dtype=torch.int32, device="cuda")
    _abi.check(_lib().cetra_net_foldpool_fwd(_stream(stream), _ptr(e.contiguous()), B, L, E,
                                             _ptr(win.trials_device(n_trial)), win.n, int(n_trial),
                                             _ptr(win.device()["q"]), _ptr(f), _ptr(arg)))
    return f, arg


def foldpool_bwd(gf, arg, win: Windows, E: int, L: int, n_trial: int, stream=None):
    """Gradient [B][L][E] of the fold-pooling features' loss w.r.t. e."""
    import torch
    B = int(gf.shape[0])
    ge = torch.empty((B, L, E), dtype=torch.float32, device="cuda")
    _abi.check(_lib().cetra_net_foldpool_bwd(_stream(stream), _ptr(gf.contiguous()), _ptr(arg.contiguous()),
                                             _ptr(win.trials_device(n_trial)), B, int(L), int(E), win.n,
                                             int(n_trial), _ptr(ge)))
    return ge
