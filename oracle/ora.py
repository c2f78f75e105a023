"""ctypes binding of the FP64 C oracle (ra_oracle.c).

TEST INFRASTRUCTURE ONLY. Only tests, the smoke check and the benchmark's CPU
baseline may use this module; the GPU library never does.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ra_oracle.c")
LIB = os.path.join(HERE, "libra_oracle.so")

HOOKEAN, FENE, HARMONIC = 0, 1, 2
QUIESCENT, UNIAXIAL, PLANAR, SHEAR = 0, 1, 2, 3
TAG_REPLICA, TAG_PARENT, TAG_EVENT = 0, 1, 2


def build(force=True):
    """Compile the oracle with gcc (plain -O2, IEEE double, no fast-math)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


class Group(ctypes.Structure):
    _fields_ = [("n_beads", ctypes.c_int32), ("n_replicas", ctypes.c_int32),
                ("spring", ctypes.c_int32), ("flow", ctypes.c_int32),
                ("H", ctypes.c_double), ("b", ctypes.c_double), ("rate", ctypes.c_double),
                ("kT", ctypes.c_double), ("zeta", ctypes.c_double), ("dt", ctypes.c_double),
                ("noise_scale", ctypes.c_double), ("rest_length", ctypes.c_double),
                ("lj_eps", ctypes.c_double), ("lj_rmin", ctypes.c_double),
                ("hi_radius", ctypes.c_double),
                ("stream_id", ctypes.c_uint32), ("pad_", ctypes.c_uint32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        dp = ctypes.POINTER(ctypes.c_double)
        L.rao_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.rao_uniform.argtypes = [ctypes.c_uint32]
        L.rao_uniform.restype = ctypes.c_double
        L.rao_uniform53.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.rao_uniform53.restype = ctypes.c_double
        L.rao_normals.argtypes = [ctypes.POINTER(ctypes.c_uint32), dp]
        L.rao_noise.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, dp]
        L.rao_normals4.argtypes = [ctypes.POINTER(ctypes.c_uint32), dp]
        L.rao_noise_mapped.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                       ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                       ctypes.c_int32, dp]
        L.rao_spring.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, dp, dp, dp, dp]
        L.rao_spring.restype = ctypes.c_int
        L.rao_flow_velocity.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        L.rao_lj.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp]
        L.rao_rpy_block.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp]
        L.rao_cholesky.argtypes = [ctypes.c_int, dp]
        L.rao_cholesky.restype = ctypes.c_int
        L.rao_lj.restype = ctypes.c_double
        L.ra_oracle_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(Group), ctypes.c_int32,
                                       ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32]
        L.ra_oracle_set_replicas.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.ra_oracle_init_chains.argtypes = [P, dp]
        L.ra_oracle_step.argtypes = [P, ctypes.c_int64]
        L.ra_oracle_n_windows.argtypes = [P]
        L.ra_oracle_n_windows.restype = ctypes.c_int64
        L.ra_oracle_total_springs.argtypes = [P]
        L.ra_oracle_total_springs.restype = ctypes.c_int64
        L.ra_oracle_average_forces.argtypes = [P, dp, dp, dp, dp]
        L.ra_oracle_bell_rates.argtypes = [P, dp, ctypes.c_int64, ctypes.c_double,
                                           ctypes.c_double, dp, dp, ctypes.POINTER(ctypes.c_uint8)]
        L.ra_oracle_backward.argtypes = [P, dp, dp, ctypes.c_double, ctypes.c_double, dp]
        L.ra_oracle_get_samples.argtypes = [P, dp, dp]
        L.ra_oracle_get_positions.argtypes = [P, dp]
        L.ra_oracle_set_tag.argtypes = [P, ctypes.c_uint32]
        L.ra_oracle_set_noise_map.argtypes = [P, ctypes.c_int32]
        L.ra_oracle_reclone.argtypes = [P, dp]
        L.ra_oracle_rsf_cycle.argtypes = [P, P, ctypes.c_int64, ctypes.c_int64]
        L.ra_oracle_block_sigma.argtypes = [P, ctypes.c_int32, dp]
        L.ra_oracle_mftu.argtypes = [P, dp, ctypes.c_int64, dp]
        L.ra_oracle_mftu_events.argtypes = [P, dp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                            ctypes.POINTER(ctypes.c_int64), dp]
        L.ra_oracle_conformation.argtypes = [P, dp, dp, dp, dp]
        L.ra_oracle_clamps.argtypes = [P, ctypes.c_int32]
        L.ra_oracle_clamps.restype = ctypes.c_int64
        L.ra_oracle_last_error.argtypes = [P]
        L.ra_oracle_last_error.restype = ctypes.c_char_p
        L.ra_oracle_destroy.argtypes = [P]
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---- primitives -----------------------------------------------------------
def philox(ctr, key):
    L = lib()
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    L.rao_philox4x32_10(c, k, o)
    return tuple(int(v) for v in o)


def uniform(x):
    return lib().rao_uniform(int(x) & 0xFFFFFFFF)


def uniform53(hi, lo):
    return lib().rao_uniform53(int(hi) & 0xFFFFFFFF, int(lo) & 0xFFFFFFFF)


def normals(words):
    w = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in words])
    o = np.zeros(3)
    lib().rao_normals(w, _dp(o))
    return o


def noise(seed, step, bead, replica, tag, group, noise_map=0):
    o = np.zeros(3)
    if noise_map:
        lib().rao_noise_mapped(seed, step, bead, replica, tag, group, noise_map, _dp(o))
    else:
        lib().rao_noise(seed, step, bead, replica, tag, group, _dp(o))
    return o


def normals4(words):
    w = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in words])
    o = np.zeros(4)
    lib().rao_normals4(w, _dp(o))
    return o


def spring(kind, H, b, kT, Q):
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    F = np.zeros(3)
    g = ctypes.c_double()
    f = ctypes.c_double()
    clamped = lib().rao_spring(kind, H, b, kT, _dp(Q), _dp(F), ctypes.byref(g), ctypes.byref(f))
    return F, g.value, f.value, bool(clamped)


def lj(u, rmin, d):
    """(U, F) of one Lennard-Jones pair, d = r_i - r_j, F the force on i."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    F = np.zeros(3)
    U = lib().rao_lj(u, rmin, _dp(d), _dp(F))
    return U, F


def rpy_block(kT, zeta, a, r):
    """RPY block D_ij (3x3) for r = r_j - r_i (Eq. 3)."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    D = np.zeros(9)
    lib().rao_rpy_block(kT, zeta, a, _dp(r), _dp(D))
    return D.reshape(3, 3)


def cholesky(A):
    """Lower Cholesky factor by the oracle's routine (None if not positive definite)."""
    L = np.ascontiguousarray(A, dtype=np.float64).copy()
    rc = lib().rao_cholesky(L.shape[0], _dp(L))
    return None if rc != 0 else L


def flow_velocity(flow, rate, r):
    r = np.ascontiguousarray(r, dtype=np.float64)
    v = np.zeros(3)
    lib().rao_flow_velocity(flow, rate, _dp(r), _dp(v))
    return v


# ---- context --------------------------------------------------------------
class OracleError(RuntimeError):
    pass


def make_groups(descs):
    arr = (Group * len(descs))()
    for i, d in enumerate(descs):
        g = arr[i]
        g.n_beads = d["n_beads"]
        g.n_replicas = d["n_replicas"]
        g.spring = d.get("spring", HOOKEAN)
        g.flow = d.get("flow", QUIESCENT)
        g.H = d.get("H", 1.0)
        g.b = d.get("b", 0.0)
        g.rate = d.get("rate", 0.0)
        g.kT = d.get("kT", 1.0)
        g.zeta = d.get("zeta", 1.0)
        g.dt = d["dt"]
        g.noise_scale = d.get("noise_scale", 1.0)
        g.rest_length = d.get("rest_length", 0.0)
        g.lj_eps = d.get("lj_eps", 0.0)
        g.lj_rmin = d.get("lj_rmin", 0.0)
        g.hi_radius = d.get("hi_radius", 0.0)
        g.stream_id = d.get("stream_id", i)
    return arr


class Oracle:
    """Context mirroring the library's calls, on host numpy arrays."""

    def __init__(self, descs, seed, sample_every, max_windows, tsf=False, tangents=False, noise_map=0):
        self.L = lib()
        self.descs = [dict(d) for d in descs]
        self._groups = make_groups(self.descs)
        self.ptr = ctypes.c_void_p()
        rc = self.L.ra_oracle_create(ctypes.byref(self.ptr), self._groups, len(descs),
                                     int(seed), int(sample_every), int(max_windows),
                                     int(bool(tsf)), int(bool(tangents)))
        if rc != 0:
            raise OracleError("ra_oracle_create failed: %d" % rc)
        self.sample_every = sample_every
        self.ranges = [(0, d["n_replicas"]) for d in descs]
        if noise_map:
            self._check(self.L.ra_oracle_set_noise_map(self.ptr, int(noise_map)), "set_noise_map")

    def _check(self, rc, what):
        if rc != 0:
            raise OracleError("%s failed (%d): %s" % (what, rc,
                              self.L.ra_oracle_last_error(self.ptr).decode()))

    def set_replicas(self, g, k_begin, k_end):
        self._check(self.L.ra_oracle_set_replicas(self.ptr, g, k_begin, k_end), "set_replicas")
        self.ranges[g] = (k_begin, k_end)

    def init_chains(self, parent_xyz):
        p = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.float64).ravel()
                                                 for x in parent_xyz]))
        self._check(self.L.ra_oracle_init_chains(self.ptr, _dp(p)), "init_chains")

    def step(self, n):
        self._check(self.L.ra_oracle_step(self.ptr, int(n)), "step")

    @property
    def n_windows(self):
        return self.L.ra_oracle_n_windows(self.ptr)

    @property
    def total_springs(self):
        return self.L.ra_oracle_total_springs(self.ptr)

    def average_forces(self, tsf=False):
        W, S = self.n_windows, self.total_springs
        mean = np.zeros((W, S))
        std = np.zeros((W, S))
        if tsf:
            tm = np.zeros((W, S))
            ts = np.zeros((W, S))
            self._check(self.L.ra_oracle_average_forces(self.ptr, _dp(mean), _dp(std),
                                                        _dp(tm), _dp(ts)), "average_forces")
            return mean, std, tm, ts
        self._check(self.L.ra_oracle_average_forces(self.ptr, _dp(mean), _dp(std), None, None),
                    "average_forces")
        return mean, std

    def bell_rates(self, mean, k0, x_dagger, events=False):
        mean = np.ascontiguousarray(mean, dtype=np.float64)
        W, S = mean.shape
        rates = np.zeros((W, S))
        rsum = np.zeros((W, len(self.descs)))
        ev = np.zeros((W, S), dtype=np.uint8) if events else None
        evp = ev.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if events else None
        self._check(self.L.ra_oracle_bell_rates(self.ptr, _dp(mean), W, k0, x_dagger,
                                                _dp(rates), _dp(rsum), evp), "bell_rates")
        return (rates, rsum, ev) if events else (rates, rsum)

    def backward(self, grad_mean, grad_rates=None, k0=0.0, x_dagger=0.0):
        gm = np.ascontiguousarray(grad_mean, dtype=np.float64)
        gr = None if grad_rates is None else np.ascontiguousarray(grad_rates, dtype=np.float64)
        out = np.zeros((len(self.descs), 3))
        self._check(self.L.ra_oracle_backward(self.ptr, _dp(gm), _dp(gr), k0, x_dagger,
                                              _dp(out)), "backward")
        return out

    def samples(self, tsf=False):
        """Per-replica tension samples, one array [W][Rsub][N-1] per group."""
        W = self.n_windows
        n = sum((e - b) * (d["n_beads"] - 1) for d, (b, e) in zip(self.descs, self.ranges))
        flat = np.zeros((W, n))
        tflat = np.zeros((W, n)) if tsf else None
        self._check(self.L.ra_oracle_get_samples(self.ptr, _dp(flat), _dp(tflat)), "get_samples")
        outs, touts, off = [], [], 0
        for d, (b, e) in zip(self.descs, self.ranges):
            m = (e - b) * (d["n_beads"] - 1)
            outs.append(flat[:, off:off + m].reshape(W, e - b, d["n_beads"] - 1))
            if tsf:
                touts.append(tflat[:, off:off + m].reshape(W, e - b, d["n_beads"] - 1))
            off += m
        return (outs, touts) if tsf else outs

    def positions(self):
        n = sum((e - b) * d["n_beads"] * 3 for d, (b, e) in zip(self.descs, self.ranges))
        flat = np.zeros(n)
        self._check(self.L.ra_oracle_get_positions(self.ptr, _dp(flat)), "get_positions")
        outs, off = [], 0
        for d, (b, e) in zip(self.descs, self.ranges):
            m = (e - b) * d["n_beads"] * 3
            outs.append(flat[off:off + m].reshape(e - b, d["n_beads"], 3))
            off += m
        return outs

    def clamps(self, g):
        return self.L.ra_oracle_clamps(self.ptr, g)

    def set_tag(self, tag):
        self._check(self.L.ra_oracle_set_tag(self.ptr, int(tag)), "set_tag")

    def reclone(self, parent_xyz):
        p = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.float64).ravel()
                                                 for x in parent_xyz]))
        self._check(self.L.ra_oracle_reclone(self.ptr, _dp(p)), "reclone")

    def rsf_cycle(self, parent, n_windows, parent_steps):
        """RSF cycle; parent is an Oracle with one replica per group."""
        self._check(self.L.ra_oracle_rsf_cycle(self.ptr, parent.ptr, int(n_windows),
                                               int(parent_steps)), "rsf_cycle")

    def block_sigma(self, block):
        sig = np.zeros((self.n_windows, self.total_springs))
        self._check(self.L.ra_oracle_block_sigma(self.ptr, int(block), _dp(sig)), "block_sigma")
        return sig

    def mftu(self, rate_sum):
        rs = np.ascontiguousarray(rate_sum, dtype=np.float64)
        out = np.zeros(len(self.descs))
        self._check(self.L.ra_oracle_mftu(self.ptr, _dp(rs), rs.shape[0], _dp(out)), "mftu")
        return out

    def mftu_events(self, rates, n_trials, max_windows):
        """(mftu [G], first window [n_trials][G]) by event sampling over the
        rate windows repeated in order."""
        r = np.ascontiguousarray(rates, dtype=np.float64)
        out = np.zeros(len(self.descs))
        first = np.zeros((n_trials, len(self.descs)), dtype=np.int64)
        self._check(self.L.ra_oracle_mftu_events(self.ptr, _dp(r), r.shape[0], int(n_trials), int(max_windows),
                                                 first.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                                 _dp(out)), "mftu_events")
        return out, first

    def conformation(self, per_bead=False):
        """(dbar [Rsim][3], rg2 [Rsim][3], src_rg2 [G][3][, d_bead [Rsim][N][3] per group])."""
        nr = sum(e - b for b, e in self.ranges)
        nb = sum((e - b) * d["n_beads"] for d, (b, e) in zip(self.descs, self.ranges))
        dbar = np.zeros((nr, 3))
        rg2 = np.zeros((nr, 3))
        src = np.zeros((len(self.descs), 3))
        db = np.zeros((nb, 3)) if per_bead else None
        self._check(self.L.ra_oracle_conformation(self.ptr, _dp(dbar), _dp(db), _dp(rg2), _dp(src)),
                    "conformation")
        return (dbar, rg2, src, db) if per_bead else (dbar, rg2, src)

    def close(self):
        if self.ptr:
            self.L.ra_oracle_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
