"""Thin Python binding of the C ABI in include/ra.h (libra.so, built in-tree).

Argument marshalling only: every step of the path runs in the HIP kernels of
libra.so. PyTorch provides device memory (tensors) and the stream. There is
no fallback: if the library is missing or fails to load, this module raises.
"""
import ctypes
import os

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libra.so")

RA_OK, RA_EINVAL, RA_ENOMEM, RA_EDEVICE, RA_EUNSTABLE, RA_ESTATE = 0, -1, -2, -3, -4, -5
HOOKEAN, FENE, HARMONIC = 0, 1, 2
CKPT_AUTO = -1
QUIESCENT, UNIAXIAL, PLANAR, SHEAR = 0, 1, 2, 3
_NAMES = {RA_EINVAL: "RA_EINVAL", RA_ENOMEM: "RA_ENOMEM", RA_EDEVICE: "RA_EDEVICE",
          RA_EUNSTABLE: "RA_EUNSTABLE", RA_ESTATE: "RA_ESTATE"}

# Every symbol include/ra.h declares.
EXPORTS = ["ra_create", "ra_init_chains", "ra_step", "ra_average_forces", "ra_bell_rates",
           "ra_backward", "ra_reclone", "ra_rsf_cycle", "ra_block_sigma", "ra_mftu", "ra_mftu_events",
           "ra_conformation",
           "ra_sync_status", "ra_guard_counts", "ra_get_samples", "ra_get_bonds",
           "ra_checkpoint_interval", "ra_tile_info", "ra_debug_noise", "ra_run_static", "ra_last_error",
           "ra_destroy"]


class RAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_NAMES.get(code, str(code)), msg))
        self.code = code


class ChainDesc(ctypes.Structure):
    _fields_ = [("n_beads", ctypes.c_int32), ("n_replicas", ctypes.c_int32),
                ("spring", ctypes.c_int32), ("flow", ctypes.c_int32),
                ("H", ctypes.c_double), ("b", ctypes.c_double), ("rate", ctypes.c_double),
                ("kT", ctypes.c_double), ("zeta", ctypes.c_double), ("dt", ctypes.c_double),
                ("noise_scale", ctypes.c_double), ("rest_length", ctypes.c_double),
                ("lj_eps", ctypes.c_double), ("lj_rmin", ctypes.c_double),
                ("hi_radius", ctypes.c_double),
                ("stream_id", ctypes.c_uint32), ("pad_", ctypes.c_uint32)]


class RunDesc(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("precision", ctypes.c_int32),
                ("sample_every", ctypes.c_int32), ("max_windows", ctypes.c_int32),
                ("tsf", ctypes.c_int32), ("checkpoint_every", ctypes.c_int32),
                ("max_steps", ctypes.c_int32), ("plain", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("tile_policy", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32), ("noise_tag", ctypes.c_int32),
                ("noise_map", ctypes.c_int32)]


assert ctypes.sizeof(ChainDesc) == 112 and ctypes.sizeof(RunDesc) == 56

_lib = None


def library():
    """Load libra.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libra.so not found at %s: build it with "
                           "`python -m paper_2206_05851_amd.build` (no CPU fallback exists)" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    sig = {
        "ra_create": [ctypes.POINTER(P), ctypes.POINTER(ChainDesc), i32, ctypes.POINTER(RunDesc), P],
        "ra_init_chains": [P, P],
        "ra_step": [P, i64],
        "ra_average_forces": [P, P, P, P, P, ctypes.POINTER(i64)],
        "ra_bell_rates": [P, P, i64, dbl, dbl, P, P, P],
        "ra_backward": [P, P, P, P, dbl, dbl, P],
        "ra_reclone": [P, P],
        "ra_rsf_cycle": [P, P, i64, i64],
        "ra_block_sigma": [P, i32, P],
        "ra_mftu": [P, P, i64, P],
        "ra_mftu_events": [P, P, i64, i32, i64, P, P],
        "ra_conformation": [P, P, P, P, P],
        "ra_sync_status": [P],
        "ra_guard_counts": [P, ctypes.POINTER(i64)],
        "ra_get_samples": [P, P, P],
        "ra_get_bonds": [P, P],
        "ra_checkpoint_interval": [P, ctypes.POINTER(i32)],
        "ra_tile_info": [P, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "ra_debug_noise": [P, i64, u64, P, P, P, P],
        "ra_run_static": [ctypes.POINTER(ChainDesc), ctypes.POINTER(RunDesc), P, i64, P, P, P],
        "ra_destroy": [P],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = None if name == "ra_destroy" else ctypes.c_int
    L.ra_last_error.argtypes = [P]
    L.ra_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _need(t, name, shape, dtype=torch.float64):
    """Check a tensor's shape and dtype before its pointer crosses the C ABI,
    which has no sizes to check against (a short buffer would be read or
    written past its end on the device)."""
    if t is None:
        return None
    if not torch.is_tensor(t) or tuple(t.shape) != tuple(shape) or t.dtype != dtype:
        got = (t.dtype, tuple(t.shape)) if torch.is_tensor(t) else type(t).__name__
        raise ValueError("%s: expected %s of shape %s, got %s" % (name, dtype, tuple(shape), got))
    return t


def _stream_handle(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_desc(d, index):
    c = ChainDesc()
    c.n_beads = int(d["n_beads"])
    c.n_replicas = int(d["n_replicas"])
    c.spring = int(d.get("spring", HOOKEAN))
    c.flow = int(d.get("flow", QUIESCENT))
    c.H = float(d.get("H", 1.0))
    c.b = float(d.get("b", 0.0))
    c.rate = float(d.get("rate", 0.0))
    c.kT = float(d.get("kT", 1.0))
    c.zeta = float(d.get("zeta", 1.0))
    c.dt = float(d["dt"])
    c.noise_scale = float(d.get("noise_scale", 1.0))
    c.rest_length = float(d.get("rest_length", 0.0))
    c.lj_eps = float(d.get("lj_eps", 0.0))
    c.lj_rmin = float(d.get("lj_rmin", 0.0))
    c.hi_radius = float(d.get("hi_radius", 0.0))
    c.stream_id = int(d.get("stream_id", index))
    return c


def debug_noise(counters, seed, words=True, n32=True, n64=True, stream=None):
    """Philox words and FP32/FP64 normals for device int32 counters [n,4]."""
    L = library()
    n = counters.shape[0]
    _need(counters, "counters", (n, 4), torch.int32)
    dev = counters.device
    w = torch.empty((n, 4), dtype=torch.int32, device=dev) if words else None
    a = torch.empty((n, 3), dtype=torch.float32, device=dev) if n32 else None
    b = torch.empty((n, 3), dtype=torch.float64, device=dev) if n64 else None
    rc = L.ra_debug_noise(_ptr(counters.contiguous()), n, int(seed), _ptr(w), _ptr(a), _ptr(b),
                          _stream_handle(stream))
    if rc != RA_OK:
        raise RAError(rc, L.ra_last_error(None).decode())
    return w, a, b


def run_static(group, seed, n_steps, sample_every, parent, precision=32, noise_map=0, tile_policy=0,
                waves_per_block=0, stream=None, out=None):
    """ra_run_static: clone, n_steps steps and replica averages of one chain
    group with the library's static scratch array (no device allocation in
    the library). parent: device FP64 tensor of N*3 values. Returns (mean,
    std), device FP64 [W, N-1] (out=(mean, std) reuses caller buffers)."""
    L = library()
    W = n_steps // sample_every
    nm1 = int(group["n_beads"]) - 1
    _need(parent.reshape(-1), "parent", (3 * int(group["n_beads"]),))
    if out is None:
        mean = torch.empty((W, nm1), dtype=torch.float64, device=parent.device)
        std = torch.empty((W, nm1), dtype=torch.float64, device=parent.device)
    else:
        mean, std = out
        _need(mean, "out[0]", (W, nm1))
        _need(std, "out[1]", (W, nm1))
    desc = make_desc(group, 0)
    run = RunDesc(seed=int(seed), precision=precision, sample_every=sample_every, max_windows=W,
                  tile_policy=tile_policy, waves_per_block=waves_per_block, noise_map=noise_map)
    par = parent.contiguous()
    rc = L.ra_run_static(ctypes.byref(desc), ctypes.byref(run), _ptr(par), int(n_steps), _ptr(mean), _ptr(std),
                         _stream_handle(stream))
    if rc != RA_OK:
        raise RAError(rc, L.ra_last_error(None).decode())
    return mean, std


class Replicas:
    """A context: groups of replicas of parent chains on one GPU."""

    def __init__(self, groups, seed, precision=32, sample_every=100, max_windows=100, tsf=False,
                 checkpoint_every=0, max_steps=0, plain=False, use_graph=False, tile_policy=0,
                 waves_per_block=0, noise_tag=0, noise_map=0, device=None, stream=None):
        self.L = library()
        self.groups = [dict(g) for g in groups]
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream
        self.precision = precision
        self.sample_every = sample_every
        self.seed = seed
        arr = (ChainDesc * len(groups))(*[make_desc(g, i) for i, g in enumerate(groups)])
        run = RunDesc(seed=int(seed), precision=precision, sample_every=sample_every,
                      max_windows=max_windows, tsf=int(bool(tsf)), checkpoint_every=checkpoint_every,
                      max_steps=max_steps, plain=int(bool(plain)), use_graph=int(bool(use_graph)),
                      tile_policy=tile_policy, waves_per_block=waves_per_block, noise_tag=noise_tag,
                      noise_map=noise_map)
        self._descs = arr
        self.ptr = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.L.ra_create(ctypes.byref(self.ptr), arr, len(groups), ctypes.byref(run),
                                  _stream_handle(stream))
        if rc != RA_OK:
            raise RAError(rc, self.L.ra_last_error(None).decode())
        self.n_springs = sum(g["n_beads"] - 1 for g in groups)
        self.n_samples = sum(g["n_replicas"] * (g["n_beads"] - 1) for g in groups)
        self.n_bond_values = 3 * self.n_samples
        self.n_windows = 0
        self.tsf = bool(tsf)

    def _check(self, rc):
        if rc != RA_OK:
            raise RAError(rc, self.L.ra_last_error(self.ptr).decode())

    # A context may run on its own stream; tensors are made and read on the
    # caller's current stream. Order the two around every call that takes or
    # returns tensors.
    def _enter(self):
        if self.stream is not None:
            self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        if self.stream is not None:
            torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def _dev(self, shape, dtype=torch.float64):
        return torch.empty(shape, dtype=dtype, device=self.device)

    def init_chains(self, parents):
        """parents: a device FP64 tensor with N_g*3 values per group, or a list of
        [N_g, 3] arrays (copied to the device first)."""
        if not torch.is_tensor(parents):
            flat = torch.cat([torch.as_tensor(p, dtype=torch.float64).reshape(-1) for p in parents])
            parents = flat.to(self.device)
        n_xyz = sum(3 * g["n_beads"] for g in self.groups)
        _need(parents.reshape(-1), "parents", (n_xyz,))
        self._parents = parents.contiguous()
        self._enter()
        self._check(self.L.ra_init_chains(self.ptr, _ptr(self._parents)))
        self.n_windows = 0

    def step(self, n):
        self._check(self.L.ra_step(self.ptr, int(n)))

    def average_forces(self, tsf=False, out=None):
        W = ctypes.c_int64()
        self._check(self.L.ra_average_forces(self.ptr, None, None, None, None, ctypes.byref(W)))
        self.n_windows = W.value
        if out is None:
            mean = self._dev((W.value, self.n_springs))
            std = self._dev((W.value, self.n_springs))
        else:
            mean, std = out
            _need(mean, "out[0]", (W.value, self.n_springs))
            _need(std, "out[1]", (W.value, self.n_springs))
        tm = self._dev((W.value, self.n_springs)) if tsf else None
        ts = self._dev((W.value, self.n_springs)) if tsf else None
        self._enter()
        self._check(self.L.ra_average_forces(self.ptr, _ptr(mean), _ptr(std), _ptr(tm), _ptr(ts), None))
        self._leave()
        return (mean, std, tm, ts) if tsf else (mean, std)

    def _windows(self):
        W = ctypes.c_int64()
        self._check(self.L.ra_average_forces(self.ptr, None, None, None, None, ctypes.byref(W)))
        return W.value

    def bell_rates(self, mean, k0, x_dagger, events=False):
        W = mean.shape[0]
        _need(mean, "mean", (W, self.n_springs))
        rates = self._dev((W, self.n_springs))
        rsum = self._dev((W, len(self.groups)))
        ev = self._dev((W, self.n_springs), torch.uint8) if events else None
        self._enter()
        self._check(self.L.ra_bell_rates(self.ptr, _ptr(mean), W, float(k0), float(x_dagger),
                                         _ptr(rates), _ptr(rsum), _ptr(ev)))
        self._leave()
        return (rates, rsum, ev) if events else (rates, rsum)

    def backward(self, mean, grad_mean, grad_rates=None, k0=0.0, x_dagger=0.0):
        out = self._dev((len(self.groups), 3))
        shape = (self._windows(), self.n_springs)
        gm = _need(grad_mean, "grad_mean", shape)
        gr = _need(grad_rates, "grad_rates", shape)
        if gr is not None:
            _need(mean, "mean", shape)
        gm = gm.contiguous() if gm is not None else None
        gr = gr.contiguous() if gr is not None else None
        self._enter()
        self._check(self.L.ra_backward(self.ptr, _ptr(mean), _ptr(gm), _ptr(gr), float(k0),
                                       float(x_dagger), _ptr(out)))
        self._leave()
        return out

    def reclone(self, parent):
        """RSF re-clone (Sec. II) from another context's current chains."""
        self._check(self.L.ra_reclone(self.ptr, parent.ptr))

    def rsf_cycle(self, parent, n_windows, parent_steps):
        """RSF sampling cycle (Sec. II) driven by a parent context."""
        self._check(self.L.ra_rsf_cycle(self.ptr, parent.ptr, int(n_windows), int(parent_steps)))

    def block_sigma(self, block):
        """Spread of the RSF estimate over blocks of `block` replicas, [W, springs]."""
        W = ctypes.c_int64()
        self._check(self.L.ra_average_forces(self.ptr, None, None, None, None, ctypes.byref(W)))
        out = self._dev((W.value, self.n_springs))
        self._enter()
        self._check(self.L.ra_block_sigma(self.ptr, int(block), _ptr(out)))
        self._leave()
        return out

    def mftu(self, rate_sum):
        """1 / (window mean of the per-chain total rate), one value per group."""
        out = self._dev((len(self.groups),))
        _need(rate_sum, "rate_sum", (rate_sum.shape[0], len(self.groups)))
        rs = rate_sum.contiguous()
        self._enter()
        self._check(self.L.ra_mftu(self.ptr, _ptr(rs), rs.shape[0], _ptr(out)))
        self._leave()
        return out

    def mftu_events(self, rates, n_trials, max_windows):
        """(mftu [G], first window [n_trials, G] (int64, -1 = censored)) by
        sampling unfolding events over the rate windows repeated in order."""
        W = rates.shape[0]
        _need(rates, "rates", (W, self.n_springs))
        out = self._dev((len(self.groups),))
        first = self._dev((int(n_trials), len(self.groups)), torch.int64)
        r = rates.contiguous()
        self._enter()
        self._check(self.L.ra_mftu_events(self.ptr, _ptr(r), W, int(n_trials), int(max_windows), _ptr(first),
                                          _ptr(out)))
        self._leave()
        return out, first

    def conformation(self, per_bead=False):
        """(dbar [sum R][3], rg2 [sum R][3], src_rg2 [G][3][, d_bead [sum R N][3]]) (Eq. 5)."""
        nr = sum(g["n_replicas"] for g in self.groups)
        nb = sum(g["n_replicas"] * g["n_beads"] for g in self.groups)
        dbar = self._dev((nr, 3))
        rg2 = self._dev((nr, 3))
        src = self._dev((len(self.groups), 3))
        db = self._dev((nb, 3)) if per_bead else None
        self._enter()
        self._check(self.L.ra_conformation(self.ptr, _ptr(dbar), _ptr(db), _ptr(rg2), _ptr(src)))
        self._leave()
        return (dbar, rg2, src, db) if per_bead else (dbar, rg2, src)

    def sync_status(self):
        self._check(self.L.ra_sync_status(self.ptr))

    def guard_counts(self):
        out = (ctypes.c_int64 * len(self.groups))()
        self._check(self.L.ra_guard_counts(self.ptr, out))
        return [int(v) for v in out]

    def samples(self, tsf=False):
        """Per-replica samples, one tensor [W, R_g, N_g-1] per group."""
        W = ctypes.c_int64()
        self._check(self.L.ra_average_forces(self.ptr, None, None, None, None, ctypes.byref(W)))
        flat = self._dev((W.value, self.n_samples))
        tflat = self._dev((W.value, self.n_samples)) if tsf else None
        self._enter()
        self._check(self.L.ra_get_samples(self.ptr, _ptr(flat), _ptr(tflat)))
        self._leave()
        outs, touts, off = [], [], 0
        for g in self.groups:
            m = g["n_replicas"] * (g["n_beads"] - 1)
            outs.append(flat[:, off:off + m].reshape(W.value, g["n_replicas"], g["n_beads"] - 1))
            if tsf:
                touts.append(tflat[:, off:off + m].reshape(W.value, g["n_replicas"], g["n_beads"] - 1))
            off += m
        return (outs, touts) if tsf else outs

    def bonds(self):
        """Current bond vectors, one tensor [R_g, N_g-1, 3] per group (FP64)."""
        flat = self._dev((self.n_bond_values,))
        self._enter()
        self._check(self.L.ra_get_bonds(self.ptr, _ptr(flat)))
        self._leave()
        outs, off = [], 0
        for g in self.groups:
            m = g["n_replicas"] * (g["n_beads"] - 1) * 3
            outs.append(flat[off:off + m].reshape(g["n_replicas"], g["n_beads"] - 1, 3))
            off += m
        return outs

    def checkpoint_interval(self):
        """Steps between kept states (CKPT_AUTO resolved; 0: no checkpoints)."""
        k = ctypes.c_int32()
        self._check(self.L.ra_checkpoint_interval(self.ptr, ctypes.byref(k)))
        return k.value

    def tile_info(self):
        """(beads per lane per group, replicas per wave per group)."""
        G = len(self.groups)
        M = (ctypes.c_int32 * G)()
        P = (ctypes.c_int32 * G)()
        self._check(self.L.ra_tile_info(self.ptr, M, P, None))
        return list(M), list(P)

    def kernel_family(self):
        """2 = pair kernel, 3 = HI kernel, 4 / 16 = one-wave families (1-4 and 6-16
        beads per lane), 0 = plain path."""
        G = len(self.groups)
        M = (ctypes.c_int32 * G)()
        P = (ctypes.c_int32 * G)()
        f = ctypes.c_int32()
        self._check(self.L.ra_tile_info(self.ptr, M, P, ctypes.byref(f)))
        return f.value

    def close(self):
        if self.ptr:
            self.L.ra_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ReplicaAverage(torch.autograd.Function):
    """(rate, H, b) per group -> (replica-mean tension profile, Bell rates).

    Forward: clone, run all steps, average, Bell rates (all on the GPU).
    Backward: the pathwise adjoint with the noise held fixed (ra_backward).
    params: CPU FP64 tensor [n_groups, 3]; the other arguments are fixed.
    """

    @staticmethod
    def forward(ctx, params, groups, parents, n_steps, seed, sample_every, k0, x_dagger,
                checkpoint_every=CKPT_AUTO):
        gs = []
        for g, p in zip(groups, params.detach().cpu().double().tolist()):
            d = dict(g)
            d["rate"], d["H"], d["b"] = p
            gs.append(d)
        rep = Replicas(gs, seed, precision=32, sample_every=sample_every,
                       max_windows=n_steps // sample_every, checkpoint_every=checkpoint_every,
                       max_steps=n_steps)
        rep.init_chains(parents)
        rep.step(n_steps)
        mean, _ = rep.average_forces()
        rates, _ = rep.bell_rates(mean, k0, x_dagger)
        ctx.rep, ctx.k0, ctx.x_dagger = rep, k0, x_dagger
        ctx.save_for_backward(mean)
        ctx.param_device = params.device
        return mean, rates

    @staticmethod
    def backward(ctx, grad_mean, grad_rates):
        (mean,) = ctx.saved_tensors
        g = ctx.rep.backward(mean, grad_mean, grad_rates, ctx.k0, ctx.x_dagger)
        ctx.rep.close()
        return (g.to(ctx.param_device),) + (None,) * 8
