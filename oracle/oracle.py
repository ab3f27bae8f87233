"""ctypes wrapper of the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  The product path never imports this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("JENGA_ORACLE_LIB", os.path.join(HERE, "liboracle.so"))
SRC = os.path.join(HERE, "jenga_oracle.c")
SRCS = [SRC, os.path.join(HERE, "episode_oracle.c")]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, -O2, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, *SRCS, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(C.Structure):
    _fields_ = [("gravity", C.c_double * 3), ("dt", C.c_double), ("restitution", C.c_double),
                ("beta", C.c_double), ("slop", C.c_double), ("margin", C.c_double),
                ("n_sub", C.c_int32), ("iters", C.c_int32), ("warm_start", C.c_int32), ("mlp_iters", C.c_int32),
                ("fallback_tau", C.c_double), ("mlp", C.POINTER(C.c_double)), ("friction_cone", C.c_int32),
                ("restitution_bias", C.c_int32), ("manifold_mode", C.c_int32), ("mega_bodies", C.c_int32),
                ("colour_partition", C.c_int32), ("_pad", C.c_int32)]


NFEAT, HIDDEN, FEAT_RECORD = 24, 128, 30
MLP_SIZE = 24 * 128 + 128 + 128 * 128 + 128 + 128 * 3 + 3 + 24 + 24


class Push(C.Structure):
    _fields_ = [("body", C.c_int32), ("start", C.c_int32), ("steps", C.c_int32), ("_pad", C.c_int32),
                ("force", C.c_double * 3), ("withdraw", C.c_double), ("x0", C.c_double * 3)]


class Manifold(C.Structure):
    _fields_ = [("a", C.c_int32), ("b", C.c_int32), ("colour", C.c_int32), ("npts", C.c_int32),
                ("axis", C.c_int32), ("band", C.c_int32), ("slot", C.c_int32 * 4),
                ("normal", C.c_double * 3), ("t1", C.c_double * 3), ("t2", C.c_double * 3),
                ("depth", C.c_double), ("sigma", C.c_double),
                ("point", (C.c_double * 3) * 4), ("lam", (C.c_double * 3) * 4), ("k", (C.c_double * 3) * 4),
                ("vbias", C.c_double * 4), ("k12", C.c_double * 4)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("candidates", C.c_int64), ("manifolds", C.c_int64),
                ("points", C.c_int64), ("contact_iters", C.c_int64), ("fallbacks", C.c_int64), ("colours", C.c_int32),
                ("error", C.c_int32), ("res_rms", C.c_double), ("res_max", C.c_double)]


class EpisodeParams(C.Structure):
    _fields_ = [("fd", C.c_double), ("ek_collapse", C.c_double), ("theta_deg", C.c_double),
                ("ek_rest", C.c_double), ("eps", C.c_double), ("rest_steps", C.c_int32), ("_pad", C.c_int32)]


class EpisodeMetrics(C.Structure):
    _fields_ = [("ek", C.c_double), ("dx_max", C.c_double), ("theta_max", C.c_double), ("margin", C.c_double),
                ("com", C.c_double * 2), ("n_support", C.c_int32), ("c_d", C.c_int32), ("c_k", C.c_int32),
                ("c_theta", C.c_int32)]


class EpisodeState(C.Structure):
    _fields_ = [("collapsed", C.c_int32), ("done", C.c_int32), ("collapse_step", C.c_int32),
                ("rest_step", C.c_int32), ("imbalance", C.c_double), ("last", EpisodeMetrics)]


def episode_params(fd=0.5, ek_collapse=5e-5, theta_deg=30.0, ek_rest=1e-7, eps=2e-3, rest_steps=400):
    """Thresholds of Eq. (collapse), the support epsilon of Eq. (stability) and the rest rule of
    Sec. "Full Floor Contact Simulation" (the paper's values by default)."""
    E = EpisodeParams()
    E.fd, E.ek_collapse, E.theta_deg, E.ek_rest, E.eps, E.rest_steps = fd, ek_collapse, theta_deg, ek_rest, eps, \
        int(rest_steps)
    return E


class SatResult(C.Structure):
    _fields_ = [("collide", C.c_int32), ("axis", C.c_int32), ("band", C.c_int32), ("_pad", C.c_int32),
                ("depth", C.c_double), ("sigma", C.c_double), ("normal", C.c_double * 3)]


BAND_SEPARATION, BAND_NORMAL, BAND_CROSS, BAND_CLIP, BAND_GROUND, BAND_EMPTY = 1, 2, 4, 8, 16, 32

_lib = None
_lock = threading.Lock()
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                build()
            L = C.CDLL(LIB_PATH)
            L.or_quat_to_rot.argtypes = [_dp, _dp]
            L.or_box_inertia.argtypes = [C.c_double, _dp, _dp]
            L.or_sat.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp, C.POINTER(SatResult)]
            L.or_sat_ex.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp, C.c_int32, C.POINTER(SatResult)]
            L.or_manifold_box.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp, _dp, C.c_double, C.POINTER(Manifold)]
            L.or_manifold_box.restype = C.c_int
            L.or_manifold_refface.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp, _dp, C.c_double, C.c_int,
                                              C.POINTER(Manifold)]
            L.or_manifold_refface.restype = C.c_int
            L.or_manifold_ground.argtypes = [_dp, _dp, _dp, C.POINTER(Manifold)]
            L.or_manifold_ground.restype = C.c_int
            L.or_pgs.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp, C.c_int, C.POINTER(Manifold), C.c_double,
                                 C.c_double, C.c_int, _dp]
            L.or_pgs_ex.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp, C.c_int, C.POINTER(Manifold), C.c_double,
                                    C.c_double, C.c_int, C.c_int, C.c_int, _dp]
            L.or_step_tower.argtypes = [C.POINTER(Params), C.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _u8p, C.c_double,
                                        C.c_int, C.POINTER(Push), C.POINTER(C.c_int64), C.c_int,
                                        C.POINTER(Manifold), C.c_int, C.POINTER(Manifold), C.c_int,
                                        C.POINTER(C.c_int), C.POINTER(Stats), C.c_void_p, C.c_int,
                                        C.POINTER(C.c_int)]
            L.or_step_tower.restype = C.c_int
            L.or_bf16.argtypes = [C.c_double]
            L.or_bf16.restype = C.c_double
            L.or_mlp_forward.argtypes = [_dp, _dp, _dp]
            L.or_broadphase.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _u8p, C.c_double, _i32p, C.c_int]
            L.or_broadphase.restype = C.c_int
            L.or_episode_eval.argtypes = [C.POINTER(EpisodeParams), C.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _u8p, _dp,
                                          C.POINTER(EpisodeMetrics)]
            L.or_step_episode.argtypes = [C.POINTER(Params), C.POINTER(EpisodeParams), C.c_int, _dp, _dp, _dp, _dp,
                                          _dp, _dp, _u8p, C.c_double, C.c_int, C.POINTER(Push),
                                          C.POINTER(C.c_int64), _dp, C.POINTER(EpisodeState),
                                          C.POINTER(Manifold), C.c_int, C.POINTER(Manifold), C.c_int,
                                          C.POINTER(C.c_int), C.POINTER(Stats)]
            L.or_step_episode.restype = C.c_int
            _lib = L
    return _lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a.reshape(shape) if shape is not None else a


def make_params(p: dict, warm_start: int = 0, mlp=None, mlp_iters: int = 0,
                fallback_tau: float = float("inf")) -> Params:
    """Solver parameters.  ``mlp`` (flat float64, MLP_SIZE, bf16-rounded) is kept alive by the
    caller; warm_start 2 uses it with ``mlp_iters`` sweeps and the residual fallback."""
    P = Params()
    P.gravity[:] = [float(g) for g in p["gravity"]]
    P.dt = float(p["dt"])
    P.restitution = float(p["restitution"])
    P.beta = float(p["beta"])
    P.slop = float(p["slop"])
    P.margin = float(p["margin"])
    P.n_sub = int(p["n_sub"])
    P.iters = int(p["iters"])
    P.warm_start = int(warm_start)
    P.mlp_iters = int(mlp_iters)
    P.fallback_tau = float(fallback_tau)
    P.friction_cone = int(p.get("friction_cone", 0))
    P.restitution_bias = int(p.get("restitution_bias", 0))
    P.manifold_mode = int(p.get("manifold_mode", 0))
    P.mega_bodies = int(p.get("mega_bodies", 0))
    P.colour_partition = int(p.get("colour_partition", 0))
    if mlp is not None:
        assert mlp.dtype == np.float64 and mlp.flags.c_contiguous and mlp.size == MLP_SIZE
        P.mlp = mlp.ctypes.data_as(C.POINTER(C.c_double))
    return P


def bf16(x: float) -> float:
    return lib().or_bf16(float(x))


def mlp_forward(mlp, f) -> np.ndarray:
    """Network output (3,) for one feature vector (24,), FP64 with bf16-rounded layer inputs."""
    y = np.zeros(3)
    lib().or_mlp_forward(_f64(mlp), _f64(f, NFEAT), y)
    return y


# ---------------------------------------------------------------------------------------------
# stage functions
# ---------------------------------------------------------------------------------------------

def quat_to_rot(q) -> np.ndarray:
    R = np.zeros(9)
    lib().or_quat_to_rot(_f64(q, 4), R)
    return R.reshape(3, 3)


def box_inertia(m, he) -> np.ndarray:
    I = np.zeros(3)
    lib().or_box_inertia(float(m), _f64(he, 3), I)
    return I


def sat(heA, xA, qA, heB, xB, qB, prefer_face=False) -> SatResult:
    """15-axis SAT; prefer_face: the reference-face variant's choice of the normal."""
    r = SatResult()
    lib().or_sat_ex(_f64(heA, 3), _f64(xA, 3), _f64(qA, 4), _f64(heB, 3), _f64(xB, 3), _f64(qB, 4),
                    int(bool(prefer_face)), C.byref(r))
    return r


def manifold_box(heA, xA, qA, heB, xB, qB, normal, depth) -> Manifold:
    m = Manifold()
    lib().or_manifold_box(_f64(heA, 3), _f64(xA, 3), _f64(qA, 4), _f64(heB, 3), _f64(xB, 3), _f64(qB, 4),
                          _f64(normal, 3), float(depth), C.byref(m))
    return m


def manifold_refface(heA, xA, qA, heB, xB, qB, normal, depth, axis) -> Manifold:
    """Reference-face clipping manifold of a colliding pair (axis: its SAT axis 0..14)."""
    m = Manifold()
    lib().or_manifold_refface(_f64(heA, 3), _f64(xA, 3), _f64(qA, 4), _f64(heB, 3), _f64(xB, 3), _f64(qB, 4),
                              _f64(normal, 3), float(depth), int(axis), C.byref(m))
    return m


def manifold_ground(he, x, q):
    m = Manifold()
    hit = lib().or_manifold_ground(_f64(he, 3), _f64(x, 3), _f64(q, 4), C.byref(m))
    return m if hit else None


def pgs(invm, Iinv, x, v, w, manifolds, mu, restitution, iters, cone=False, bias=False):
    """PGS on explicit manifolds (processed in list order). Returns (v, w, manifolds, residual).
    cone: the tangent pair projected onto the friction disc; bias: pre-solve restitution targets."""
    nb = len(invm)
    v = _f64(v, (nb, 3)).copy()
    w = _f64(w, (nb, 3)).copy()
    arr = (Manifold * max(1, len(manifolds)))()
    for i, m in enumerate(manifolds):
        arr[i] = m
    res = np.zeros(2)
    lib().or_pgs_ex(nb, _f64(invm, nb), _f64(Iinv, (nb, 9)), _f64(x, (nb, 3)), v, w, len(manifolds), arr,
                    float(mu), float(restitution), int(bool(cone)), int(bool(bias)), int(iters), res)
    return v, w, [arr[i] for i in range(len(manifolds))], res


def broadphase(he, mass, x, q, active, margin):
    nb = len(mass)
    cap = nb * (nb + 1) // 2 + 1
    pairs = np.zeros(2 * cap, np.int32)
    n = lib().or_broadphase(nb, _f64(he, (nb, 3)), _f64(mass, nb), _f64(x, (nb, 3)), _f64(q, (nb, 4)),
                            np.ascontiguousarray(active, np.uint8), float(margin), pairs, cap)
    return pairs[:2 * n].reshape(n, 2)


def episode_eval(he, mass, x, q, v, w, active, x0, E: EpisodeParams | None = None) -> dict:
    """Eq. (stability) margin and the terms of Eq. (collapse) for one tower's state."""
    nb = len(mass)
    out = EpisodeMetrics()
    lib().or_episode_eval(C.byref(E or episode_params()), nb, _f64(he, (nb, 3)), _f64(mass, nb), _f64(x, (nb, 3)),
                          _f64(q, (nb, 4)), _f64(v, (nb, 3)), _f64(w, (nb, 3)), np.ascontiguousarray(active, np.uint8),
                          _f64(x0, (nb, 3)), C.byref(out))
    return metrics_dict(out)


def metrics_dict(m: EpisodeMetrics) -> dict:
    return dict(ek=m.ek, dx_max=m.dx_max, theta_max=m.theta_max, margin=m.margin, com=np.array(m.com[:]),
                n_support=m.n_support, c_d=bool(m.c_d), c_k=bool(m.c_k), c_theta=bool(m.c_theta))


def manifold_dict(m: Manifold) -> dict:
    n = m.npts
    return dict(a=m.a, b=m.b, colour=m.colour, npts=n, axis=m.axis, band=m.band,
                slot=np.array(m.slot[:n], np.int32),
                normal=np.array(m.normal[:]), t1=np.array(m.t1[:]), t2=np.array(m.t2[:]),
                depth=m.depth, sigma=m.sigma,
                point=np.array([m.point[i][:] for i in range(n)]).reshape(n, 3),
                lam=np.array([m.lam[i][:] for i in range(n)]).reshape(n, 3),
                k=np.array([m.k[i][:] for i in range(n)]).reshape(n, 3))


# ---------------------------------------------------------------------------------------------
# scene stepping
# ---------------------------------------------------------------------------------------------

class OracleWorld:
    """All towers of a scene, stepped tower by tower in FP64."""

    def __init__(self, scene: dict, warm_start: int = 0, params: dict | None = None, mlp=None,
                 mlp_iters: int = 0, fallback_tau: float = float("inf")):
        self.scene = scene
        self.mlp = None if mlp is None else _f64(mlp).copy()
        self.params = make_params(params or scene["params"], warm_start, self.mlp, mlp_iters, fallback_tau)
        self.features = {}
        self.ptr = np.asarray(scene["tower_ptr"], np.int64)
        self.T = int(scene["n_towers"])
        self.he = _f64(scene["half_extents"]).reshape(-1, 3).copy()
        self.mass = _f64(scene["mass"]).copy()
        self.x = _f64(scene["pos"]).reshape(-1, 3).copy()
        self.q = _f64(scene["quat"]).reshape(-1, 4).copy()
        self.v = _f64(scene["linvel"]).reshape(-1, 3).copy()
        self.w = _f64(scene["angvel"]).reshape(-1, 3).copy()
        self.active = np.ascontiguousarray(scene["active"], np.uint8).copy()
        self.mu = _f64(scene["mu"]).copy()
        self.step_counter = [C.c_int64(0) for _ in range(self.T)]
        self.stats = [Stats() for _ in range(self.T)]
        self.contacts = [None] * self.T
        self.ncontacts = [0] * self.T
        self.pushes = [[] for _ in range(self.T)]
        tower = np.repeat(np.arange(self.T), np.diff(self.ptr))
        for i in range(len(scene["push_body"])):
            b = int(scene["push_body"][i])
            t = int(tower[b])
            p = Push()
            p.body = b - int(self.ptr[t])
            p.start = int(scene["push_start"][i])
            p.steps = int(scene["push_steps"][i])
            p.force[:] = [float(f) for f in scene["push_force"][i]]
            p.withdraw = float(scene["push_withdraw"][i])
            self.pushes[t].append(p)
        self.push_arrays = []
        for t in range(self.T):
            arr = (Push * max(1, len(self.pushes[t])))()
            for i, p in enumerate(self.pushes[t]):
                arr[i] = p
            self.push_arrays.append(arr)

    def set_state(self, pos, quat, linvel, angvel):
        """Overwrite the body state and forget the previous step's impulses."""
        self.x[:] = np.asarray(pos, np.float64).reshape(-1, 3)
        self.q[:] = np.asarray(quat, np.float64).reshape(-1, 4)
        self.v[:] = np.asarray(linvel, np.float64).reshape(-1, 3)
        self.w[:] = np.asarray(angvel, np.float64).reshape(-1, 3)
        self.contacts = [None] * self.T
        self.ncontacts = [0] * self.T

    def step_tower(self, t: int, n_steps: int, record: bool = False):
        a, b = int(self.ptr[t]), int(self.ptr[t + 1])
        nb = b - a
        if nb == 0:
            self.step_counter[t].value += n_steps
            return
        # views into the global arrays (contiguous slices of C-contiguous arrays)
        x = self.x[a:b]; q = self.q[a:b]; v = self.v[a:b]; w = self.w[a:b]
        act = self.active[a:b]
        cap = 6 * nb + 8
        out = (Manifold * cap)()
        nout = C.c_int(0)
        prev = self.contacts[t]
        nprev = self.ncontacts[t]
        feat = None
        nfeat = C.c_int(0)
        if record:
            fcap = 4 * cap
            feat = np.zeros((fcap, FEAT_RECORD))
        lib().or_step_tower(C.byref(self.params), nb, self.he[a:b], self.mass[a:b], x, q, v, w, act,
                            float(self.mu[t]), len(self.pushes[t]), self.push_arrays[t],
                            C.byref(self.step_counter[t]), int(n_steps),
                            prev if prev is not None else None, int(nprev), out, cap, C.byref(nout),
                            C.byref(self.stats[t]), None if feat is None else feat.ctypes.data,
                            0 if feat is None else fcap, C.byref(nfeat))
        if record:
            self.features[t] = feat[:nfeat.value].copy()
        self.contacts[t] = out
        self.ncontacts[t] = min(nout.value, cap)

    def step(self, n_steps: int = 1, towers=None, threads: int = 1, record: bool = False):
        """Step towers; with ``record`` keep the last step's per-point feature records
        (features, k, solved impulses) in ``self.features[t]``."""
        towers = range(self.T) if towers is None else towers
        if threads <= 1:
            for t in towers:
                self.step_tower(t, n_steps, record)
        else:
            with ThreadPoolExecutor(threads) as ex:
                list(ex.map(lambda t: self.step_tower(t, n_steps, record), towers))

    # -- episodes (Sec. "Stability Detection and Collapse") --------------------------------------

    def begin_episodes(self, E: EpisodeParams | None = None):
        """Start an episode in every tower: the current positions are the reference of Eq. (collapse)'s
        displacement; no tower is collapsed."""
        self.episode_E = E or episode_params()
        self.x0 = self.x.copy()
        self.episodes = [EpisodeState() for _ in range(self.T)]
        for es in self.episodes:
            es.collapse_step = es.rest_step = -1
            es.imbalance = float("nan")

    def step_tower_episode(self, t: int, n_steps: int):
        a, b = int(self.ptr[t]), int(self.ptr[t + 1])
        nb = b - a
        es = self.episodes[t]
        if nb == 0:
            self.step_counter[t].value += n_steps
            return
        x = self.x[a:b]; q = self.q[a:b]; v = self.v[a:b]; w = self.w[a:b]
        act = self.active[a:b]
        cap = 6 * nb + 8
        for _ in range(n_steps):
            out = (Manifold * cap)()
            nout = C.c_int(0)
            prev = self.contacts[t]
            lib().or_step_episode(C.byref(self.params), C.byref(self.episode_E), nb, self.he[a:b], self.mass[a:b],
                                  x, q, v, w, act, float(self.mu[t]), len(self.pushes[t]), self.push_arrays[t],
                                  C.byref(self.step_counter[t]), self.x0[a:b], C.byref(es),
                                  prev if prev is not None else None, int(self.ncontacts[t]), out, cap,
                                  C.byref(nout), C.byref(self.stats[t]))
            if not es.done or nout.value:
                self.contacts[t] = out
                self.ncontacts[t] = min(nout.value, cap)

    def step_episodes(self, n_steps: int = 1, towers=None, threads: int = 1):
        """Step towers under the episode rules (begin_episodes first)."""
        towers = range(self.T) if towers is None else towers
        if threads <= 1:
            for t in towers:
                self.step_tower_episode(t, n_steps)
        else:
            with ThreadPoolExecutor(threads) as ex:
                list(ex.map(lambda t: self.step_tower_episode(t, n_steps), towers))

    def episode(self, t: int) -> dict:
        es = self.episodes[t]
        return dict(collapsed=bool(es.collapsed), done=bool(es.done), collapse_step=es.collapse_step,
                    rest_step=es.rest_step, imbalance=es.imbalance, **metrics_dict(es.last))

    def manifolds(self, t: int):
        arr = self.contacts[t]
        if arr is None:
            return []
        return [manifold_dict(arr[i]) for i in range(self.ncontacts[t])]

    def tower_stats(self, t: int) -> Stats:
        return self.stats[t]
