"""Python binding of the C ABI in include/jenga.h (argument marshalling only).

Every step of the simulation runs in ``libjenga.so`` on the GPU.  The functions
keep the C names (``jg_create_world``, ``jg_step_batch``, ...); ``World`` wraps a
handle for convenience.  PyTorch is only used to pick the HIP stream.

Importing this module does not need a GPU; loading the library does, and fails
loudly when ``libjenga.so`` has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjenga.so")

JG_OK, JG_EINVAL, JG_ENOMEM, JG_EDEVICE, JG_ECAPACITY, JG_ESTATE, JG_ENAN = 0, -1, -2, -3, -4, -5, -6
# device error-word bits (jg_stats.error_word)
JG_ERR_CANDIDATES, JG_ERR_MANIFOLDS, JG_ERR_COLOURS, JG_ERR_NAN = 1, 2, 4, 8
ERR_CANDIDATES, ERR_MANIFOLDS, ERR_COLOURS, ERR_NAN = 1, 2, 4, 8

EXPORTS = ["jg_default_params", "jg_create_world", "jg_destroy_world", "jg_add_boxes", "jg_set_friction",
           "jg_set_push", "jg_set_active", "jg_commit", "jg_step_batch", "jg_query_state", "jg_set_state", "jg_query_active",
           "jg_query_contacts", "jg_query_stats", "jg_query_phase_cycles", "jg_query_features", "jg_set_mlp",
           "jg_world_size", "jg_sync", "jg_device_views", "jg_body_slots", "jg_begin_episodes",
           "jg_query_episode",
           "jg_last_error", "jg_mlp_packed_bytes", "jg_mlp_pack", "jg_mlp_forward", "jg_mlp_grad_workspace_bytes",
           "jg_mlp_grad", "jg_mlp_grad_noalloc", "jg_mlp_adamw"]
MLP_PARAMS, MLP_TRAINABLE, MLP_FEATURES, FEAT_RECORD = 20147, 20099, 24, 30
PHASES = ["load/store", "forces+frames", "broad+narrow", "colouring", "manifolds", "pgs", "outputs",
          "residual", "integrate", "baumgarte"]


class jg_params(C.Structure):
    _fields_ = [("gravity", C.c_double * 3), ("dt", C.c_double), ("restitution", C.c_double),
                ("beta", C.c_double), ("slop", C.c_double), ("margin", C.c_double),
                ("n_sub", C.c_int32), ("iters", C.c_int32), ("warm_start", C.c_int32), ("device", C.c_int32),
                ("stream", C.c_void_p), ("pack_bodies", C.c_int32), ("manifolds_per_body", C.c_float),
                ("mlp_iters", C.c_int32), ("fallback_tau", C.c_double), ("record_features", C.c_int32),
                ("use_graph", C.c_int32), ("collapse_fd", C.c_double), ("collapse_ek", C.c_double),
                ("collapse_theta", C.c_double), ("rest_ek", C.c_double), ("support_eps", C.c_double),
                ("rest_steps", C.c_int32), ("friction_cone", C.c_int32), ("restitution_bias", C.c_int32),
                ("manifold_mode", C.c_int32), ("mega_bodies", C.c_int32), ("colour_partition", C.c_int32),
                ("mega_cand_per_body", C.c_float), ("small_batch", C.c_int32), ("precision", C.c_int32)]


class jg_contact(C.Structure):
    _fields_ = [("tower", C.c_int32), ("body_a", C.c_int32), ("body_b", C.c_int32), ("slot", C.c_int32),
                ("colour", C.c_int32), ("order", C.c_int32), ("point", C.c_float * 3), ("normal", C.c_float * 3),
                ("t1", C.c_float * 3), ("depth", C.c_float), ("lambda_n", C.c_float), ("lambda_t1", C.c_float),
                ("lambda_t2", C.c_float)]


class jg_stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("candidates", C.c_int64), ("manifolds", C.c_int64), ("points", C.c_int64),
                ("contact_iters", C.c_int64), ("colours", C.c_int32), ("error_word", C.c_uint32),
                ("residual_rms", C.c_double), ("residual_max", C.c_double), ("fallbacks", C.c_int64)]


class jg_episode(C.Structure):
    _fields_ = [("collapsed", C.c_int32), ("done", C.c_int32), ("collapse_step", C.c_int32),
                ("rest_step", C.c_int32), ("rounds", C.c_int32), ("torque_moves", C.c_int32),
                ("removed", C.c_int32), ("support_vertices", C.c_int32), ("ek", C.c_float), ("dx_max", C.c_float),
                ("theta_max", C.c_float), ("margin", C.c_float), ("imbalance", C.c_float),
                ("com", C.c_float * 2), ("_pad", C.c_float)]


JG_MOVE_NONE, JG_MOVE_CENTER_X, JG_MOVE_SIDE_Y, JG_MOVE_SIDE_X = -1, 0, 1, 2
JG_FP32, JG_FP64 = 0, 1

CONTACT_DTYPE = np.dtype([("tower", np.int32), ("body_a", np.int32), ("body_b", np.int32), ("slot", np.int32),
                          ("colour", np.int32), ("order", np.int32), ("point", np.float32, 3),
                          ("normal", np.float32, 3), ("t1", np.float32, 3), ("depth", np.float32),
                          ("lambda_n", np.float32), ("lambda_t1", np.float32), ("lambda_t2", np.float32)])
assert CONTACT_DTYPE.itemsize == C.sizeof(jg_contact)

_lib = None
_dp = C.POINTER(C.c_double)


def load_library(path: str = LIB_PATH):
    """Load libjenga.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python paper_2606_28394_amd/build.py` "
                          "(or __graft_entry__.build())")
    # Load torch first: libjenga.so then binds to the same HIP runtime (same soname), so the
    # streams torch hands out are valid inside the library and one runtime owns the device.
    import torch  # noqa: F401
    L = C.CDLL(path)
    L.jg_default_params.argtypes = [C.POINTER(jg_params)]
    L.jg_default_params.restype = None
    L.jg_create_world.argtypes = [C.POINTER(jg_params), C.c_int32, C.c_int32, C.POINTER(C.c_void_p)]
    L.jg_destroy_world.argtypes = [C.c_void_p]
    L.jg_add_boxes.argtypes = [C.c_void_p, C.c_int32, C.c_int32, _dp, _dp, _dp, _dp, _dp, _dp,
                               C.POINTER(C.c_int32)]
    L.jg_set_friction.argtypes = [C.c_void_p, C.c_int32, C.c_double]
    L.jg_set_push.argtypes = [C.c_void_p, C.c_int32, _dp, C.c_int32, C.c_int32, C.c_double, C.c_int32]
    L.jg_set_active.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
    L.jg_commit.argtypes = [C.c_void_p]
    L.jg_step_batch.argtypes = [C.c_void_p, C.c_int32]
    L.jg_query_state.argtypes = [C.c_void_p, C.c_int32, C.c_int32, _dp, _dp, _dp, _dp]
    L.jg_set_state.argtypes = [C.c_void_p, C.c_int32, C.c_int32, _dp, _dp, _dp, _dp]
    L.jg_query_active.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_uint8)]
    L.jg_query_contacts.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]
    L.jg_query_stats.argtypes = [C.c_void_p, C.c_int32, C.POINTER(jg_stats)]
    L.jg_query_phase_cycles.argtypes = [C.c_void_p, C.POINTER(C.c_uint64), C.c_int32]
    L.jg_query_features.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_float), C.c_int32, C.POINTER(C.c_int32)]
    L.jg_set_mlp.argtypes = [C.c_void_p, C.POINTER(C.c_float)]
    L.jg_world_size.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.jg_sync.argtypes = [C.c_void_p]
    L.jg_device_views.argtypes = [C.c_void_p] + [C.POINTER(C.c_void_p)] * 4 + [C.POINTER(C.c_int32)]
    L.jg_body_slots.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
    L.jg_begin_episodes.argtypes = [C.c_void_p]
    L.jg_query_episode.argtypes = [C.c_void_p, C.c_int32, C.POINTER(jg_episode)]
    L.jg_last_error.argtypes = []
    L.jg_last_error.restype = C.c_char_p
    vp, sz = C.c_void_p, C.c_size_t
    L.jg_mlp_packed_bytes.argtypes = [C.POINTER(sz)]
    L.jg_mlp_pack.argtypes = [vp, vp, vp]
    L.jg_mlp_forward.argtypes = [vp, vp, C.c_int32, vp, vp]
    L.jg_mlp_grad_workspace_bytes.argtypes = [C.c_int32, C.POINTER(sz)]
    L.jg_mlp_grad.argtypes = [vp, vp, vp, vp, C.c_int32, vp, vp, vp, sz, vp]
    L.jg_mlp_grad_noalloc.argtypes = [vp, vp, vp, vp, C.c_int32, vp, vp, vp]
    L.jg_mlp_adamw.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float, C.c_float, vp]
    for name in EXPORTS:
        if name not in ("jg_default_params", "jg_last_error"):
            getattr(L, name).restype = C.c_int32
    _lib = L
    return L


class JengaError(RuntimeError):
    """A failed call.  For JG_ECAPACITY / JG_ENAN from a syncing call (device error bits raised
    by earlier launches) the call did its work: ``result`` holds what it returned."""

    def __init__(self, code, msg, result=None):
        super().__init__(f"jenga error {code}: {msg}")
        self.code = code
        self.result = result


def _check(code, result=None):
    if code != JG_OK:
        raise JengaError(code, load_library().jg_last_error().decode(), result)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _arr(a, shape):
    if a is None:
        return None
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape))


# ------------------------------------------------------------------------------------------------
# thin wrappers with the C names
# ------------------------------------------------------------------------------------------------

def jg_default_params() -> jg_params:
    p = jg_params()
    load_library().jg_default_params(C.byref(p))
    return p


def jg_create_world(params: jg_params, max_towers: int, max_bodies: int) -> C.c_void_p:
    h = C.c_void_p()
    _check(load_library().jg_create_world(C.byref(params), int(max_towers), int(max_bodies), C.byref(h)))
    return h


def jg_destroy_world(h):
    _check(load_library().jg_destroy_world(h))


def jg_add_boxes(h, tower, half_extents, mass, pos, quat, linvel=None, angvel=None) -> np.ndarray:
    n = len(np.atleast_1d(mass))
    he = _arr(half_extents, (n, 3)); m = _arr(mass, (n,)); x = _arr(pos, (n, 3)); q = _arr(quat, (n, 4))
    v = _arr(linvel, (n, 3)); w = _arr(angvel, (n, 3))
    ids = np.zeros(n, np.int32)
    _check(load_library().jg_add_boxes(h, int(tower), n, _ptr(he), _ptr(m), _ptr(x), _ptr(q), _ptr(v), _ptr(w),
                                       ids.ctypes.data_as(C.POINTER(C.c_int32))))
    return ids


def jg_set_friction(h, tower, mu):
    _check(load_library().jg_set_friction(h, int(tower), float(mu)))


def jg_set_push(h, body, force, start_step, n_steps, withdraw=0.0, move=JG_MOVE_NONE):
    f = _arr(force, (3,))
    _check(load_library().jg_set_push(h, int(body), _ptr(f), int(start_step), int(n_steps), float(withdraw),
                                      int(move)))


def jg_set_active(h, body, active):
    _check(load_library().jg_set_active(h, int(body), int(bool(active))))


def jg_commit(h):
    _check(load_library().jg_commit(h))


def jg_step_batch(h, n_steps):
    _check(load_library().jg_step_batch(h, int(n_steps)))


def jg_query_state(h, first, n):
    pos = np.zeros((n, 3)); quat = np.zeros((n, 4)); v = np.zeros((n, 3)); w = np.zeros((n, 3))
    _check(load_library().jg_query_state(h, int(first), int(n), _ptr(pos), _ptr(quat), _ptr(v), _ptr(w)),
           (pos, quat, v, w))
    return pos, quat, v, w


def jg_set_state(h, first, pos=None, quat=None, linvel=None, angvel=None):
    n = None
    for a, c in ((pos, 3), (quat, 4), (linvel, 3), (angvel, 3)):
        if a is not None:
            n = np.asarray(a).size // c
    if n is None:
        return
    _check(load_library().jg_set_state(h, int(first), int(n), _ptr(_arr(pos, (n, 3))), _ptr(_arr(quat, (n, 4))),
                                       _ptr(_arr(linvel, (n, 3))), _ptr(_arr(angvel, (n, 3)))))


def jg_query_active(h, first, n):
    out = np.zeros(n, np.uint8)
    _check(load_library().jg_query_active(h, int(first), int(n), out.ctypes.data_as(C.POINTER(C.c_uint8))), out)
    return out


def jg_query_contacts(h, tower, capacity=None) -> np.ndarray:
    L = load_library()
    n = C.c_int32(0)
    if capacity is None:
        rc = L.jg_query_contacts(h, int(tower), None, 0, C.byref(n))
        if rc not in (JG_OK, JG_ECAPACITY, JG_ENAN):
            _check(rc)
        capacity = n.value
        pending = rc
    else:
        pending = JG_OK
    out = np.zeros(max(1, capacity), CONTACT_DTYPE)
    rc = L.jg_query_contacts(h, int(tower), out.ctypes.data_as(C.c_void_p), int(capacity), C.byref(n))
    res = out[:min(n.value, capacity)]
    # the size query may have found the device error bits: report them with the records
    _check(rc if rc != JG_OK else pending, res)
    return res


def jg_query_stats(h, tower=-1) -> jg_stats:
    s = jg_stats()
    _check(load_library().jg_query_stats(h, int(tower), C.byref(s)), s)
    return s


def jg_query_phase_cycles(h) -> dict:
    out = (C.c_uint64 * len(PHASES))()
    rc = load_library().jg_query_phase_cycles(h, out, len(PHASES))
    res = dict(zip(PHASES, [int(v) for v in out]))
    _check(rc, res)
    return res


def jg_query_features(h, tower=-1) -> np.ndarray:
    """Feature records (n x 30: 24 features, k[3], impulses[3]) of the last step, in contact order."""
    L = load_library()
    n = C.c_int32(0)
    pending = L.jg_query_features(h, int(tower), None, 0, C.byref(n))
    if pending not in (JG_OK, JG_ECAPACITY, JG_ENAN):
        _check(pending)
    out = np.zeros((max(1, n.value), FEAT_RECORD), np.float32)
    rc = L.jg_query_features(h, int(tower), out.ctypes.data_as(C.POINTER(C.c_float)), n.value, C.byref(n))
    res = out[:n.value]
    _check(rc if rc != JG_OK else pending, res)
    return res


def jg_set_mlp(h, params):
    p = np.ascontiguousarray(np.asarray(params, np.float32).reshape(MLP_PARAMS))
    _check(load_library().jg_set_mlp(h, p.ctypes.data_as(C.POINTER(C.c_float))))


def jg_world_size(h):
    t = C.c_int32(0); b = C.c_int32(0)
    _check(load_library().jg_world_size(h, C.byref(t), C.byref(b)))
    return t.value, b.value


def jg_sync(h):
    _check(load_library().jg_sync(h))


def jg_device_views(h):
    """Device pointers (ints) of x, q, v, angvel and the array stride (see include/jenga.h)."""
    ptrs = [C.c_void_p() for _ in range(4)]
    stride = C.c_int32(0)
    _check(load_library().jg_device_views(h, *[C.byref(p) for p in ptrs], C.byref(stride)))
    return [p.value for p in ptrs], stride.value


def jg_begin_episodes(h):
    _check(load_library().jg_begin_episodes(h))


def jg_query_episode(h, tower) -> jg_episode:
    e = jg_episode()
    _check(load_library().jg_query_episode(h, int(tower), C.byref(e)), e)
    return e


def jg_body_slots(h, first, n) -> np.ndarray:
    out = np.zeros(n, np.int32)
    _check(load_library().jg_body_slots(h, int(first), int(n), out.ctypes.data_as(C.POINTER(C.c_int32))))
    return out


def jg_last_error() -> str:
    return load_library().jg_last_error().decode()


# network entry points: device pointers (ints) and a raw stream handle

def jg_mlp_packed_bytes() -> int:
    n = C.c_size_t(0)
    _check(load_library().jg_mlp_packed_bytes(C.byref(n)))
    return n.value


def jg_mlp_pack(params_ptr, packed_ptr, stream=None):
    _check(load_library().jg_mlp_pack(params_ptr, packed_ptr, stream))


def jg_mlp_forward(packed_ptr, feats_ptr, n, y_ptr, stream=None):
    _check(load_library().jg_mlp_forward(packed_ptr, feats_ptr, int(n), y_ptr, stream))


def jg_mlp_grad_workspace_bytes(n) -> int:
    b = C.c_size_t(0)
    _check(load_library().jg_mlp_grad_workspace_bytes(int(n), C.byref(b)))
    return b.value


def jg_mlp_grad(params_ptr, packed_ptr, feats_ptr, targets_ptr, n, grad_ptr, loss_ptr, ws_ptr, ws_bytes,
                stream=None):
    _check(load_library().jg_mlp_grad(params_ptr, packed_ptr, feats_ptr, targets_ptr, int(n), grad_ptr, loss_ptr,
                                      ws_ptr, int(ws_bytes), stream))


def jg_mlp_grad_noalloc(params_ptr, packed_ptr, feats_ptr, targets_ptr, n, grad_ptr, loss_ptr, stream=None):
    _check(load_library().jg_mlp_grad_noalloc(params_ptr, packed_ptr, feats_ptr, targets_ptr, int(n), grad_ptr,
                                              loss_ptr, stream))


def jg_mlp_adamw(params_ptr, grad_ptr, m_ptr, v_ptr, step, lr, beta1, beta2, eps, weight_decay, stream=None):
    _check(load_library().jg_mlp_adamw(params_ptr, grad_ptr, m_ptr, v_ptr, int(step), float(lr), float(beta1),
                                       float(beta2), float(eps), float(weight_decay), stream))


# ------------------------------------------------------------------------------------------------
# convenience handles
# ------------------------------------------------------------------------------------------------

class Mlp:
    """Device copies of the warm-start network (torch tensors as memory): FP32 parameters,
    their packed bfloat16 form, AdamW moments and a gradient workspace."""

    def __init__(self, params, device: str = "cuda"):
        import torch
        p = torch.as_tensor(np.asarray(params, np.float32).reshape(MLP_PARAMS))
        self.torch = torch
        self.params = p.to(device).contiguous()
        self.packed = torch.zeros(jg_mlp_packed_bytes(), dtype=torch.uint8, device=device)
        self.m = torch.zeros(MLP_TRAINABLE, dtype=torch.float32, device=device)
        self.v = torch.zeros(MLP_TRAINABLE, dtype=torch.float32, device=device)
        self.grad = torch.zeros(MLP_TRAINABLE, dtype=torch.float32, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.ws = torch.zeros(0, dtype=torch.uint8, device=device)
        self.step_count = 0
        self.pack()

    def _stream(self):
        return self.torch.cuda.current_stream().cuda_stream

    def pack(self):
        jg_mlp_pack(self.params.data_ptr(), self.packed.data_ptr(), self._stream())

    def forward(self, feats):
        f = feats.contiguous()
        y = self.torch.empty((f.shape[0], 3), dtype=self.torch.float32, device=f.device)
        jg_mlp_forward(self.packed.data_ptr(), f.data_ptr(), f.shape[0], y.data_ptr(), self._stream())
        return y

    def compute_grad(self, feats, targets):
        """Gradient (JG_MLP_TRAINABLE) and loss of the mean squared error on one batch."""
        f, t = feats.contiguous(), targets.contiguous()
        need = jg_mlp_grad_workspace_bytes(f.shape[0])
        if self.ws.numel() < need:
            self.ws = self.torch.zeros(need, dtype=self.torch.uint8, device=f.device)
        jg_mlp_grad(self.params.data_ptr(), self.packed.data_ptr(), f.data_ptr(), t.data_ptr(), f.shape[0],
                    self.grad.data_ptr(), self.loss.data_ptr(), self.ws.data_ptr(), self.ws.numel(), self._stream())
        return self.grad, self.loss

    def adamw(self, lr=3e-4, betas=(0.9, 0.999), eps=1e-8, weight_decay=1e-4):
        self.step_count += 1
        jg_mlp_adamw(self.params.data_ptr(), self.grad.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                     self.step_count, lr, betas[0], betas[1], eps, weight_decay, self._stream())
        self.pack()

    def train_step(self, feats, targets, **opt):
        _, loss = self.compute_grad(feats, targets)
        self.adamw(**opt)
        return loss


def current_stream_handle():
    """The raw hipStream_t of torch's current stream (None without a GPU)."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:   # torch is optional for the binding
        pass
    return None


class World:
    """A world built from a scene dict (see workloads.py); bodies keep the scene's order."""

    def __init__(self, scene: dict, warm_start: int = 0, stream=None, device: int = 0, pack_bodies: int = 0,
                 manifolds_per_body: float = 0.0, params: dict | None = None, mlp=None, mlp_iters: int = 8,
                 fallback_tau: float = 1e30, record_features: bool = False, use_graph: bool = False,
                 small_batch: int = 0,
                 episode: dict | None = None):
        pr = params or scene["params"]
        p = jg_default_params()
        p.gravity[:] = [float(g) for g in pr["gravity"]]
        p.dt = float(pr["dt"])
        p.restitution = float(pr["restitution"])
        p.beta = float(pr["beta"])
        p.slop = float(pr["slop"])
        p.margin = float(pr["margin"])
        p.n_sub = int(pr["n_sub"])
        p.iters = int(pr["iters"])
        p.friction_cone = int(pr.get("friction_cone", 0))
        p.restitution_bias = int(pr.get("restitution_bias", 0))
        p.manifold_mode = int(pr.get("manifold_mode", 0))
        p.mega_bodies = int(pr.get("mega_bodies", 16384))
        p.colour_partition = int(pr.get("colour_partition", 1024))
        p.mega_cand_per_body = float(pr.get("mega_cand_per_body", 16.0))
        p.warm_start = int(warm_start)
        p.device = int(device)
        p.stream = stream if stream is not None else current_stream_handle()
        p.pack_bodies = int(pack_bodies)
        p.manifolds_per_body = float(manifolds_per_body)
        p.mlp_iters = int(mlp_iters)
        p.fallback_tau = float(fallback_tau)
        p.record_features = int(bool(record_features))
        p.use_graph = int(bool(use_graph))
        p.small_batch = int(small_batch)
        for k, v in (episode or {}).items():     # collapse_fd, collapse_ek, ..., rest_steps
            setattr(p, k, type(getattr(p, k))(v))
        self.params = p
        T = int(scene["n_towers"])
        ptr = np.asarray(scene["tower_ptr"])
        N = int(ptr[-1])
        self.n_towers, self.n_bodies = T, N
        self.h = jg_create_world(p, max(1, T), max(1, N))
        for t in range(T):
            a, b = int(ptr[t]), int(ptr[t + 1])
            if b > a:
                jg_add_boxes(self.h, t, scene["half_extents"][a:b], scene["mass"][a:b], scene["pos"][a:b],
                             scene["quat"][a:b], scene["linvel"][a:b], scene["angvel"][a:b])
            jg_set_friction(self.h, t, float(scene["mu"][t]))
        act = np.asarray(scene["active"])
        for i in np.nonzero(act == 0)[0]:
            jg_set_active(self.h, int(i), 0)
        moves = scene.get("push_move")
        for i in range(len(scene["push_body"])):
            jg_set_push(self.h, int(scene["push_body"][i]), scene["push_force"][i], int(scene["push_start"][i]),
                        int(scene["push_steps"][i]), float(scene["push_withdraw"][i]),
                        JG_MOVE_NONE if moves is None else int(moves[i]))
        if mlp is not None:
            jg_set_mlp(self.h, mlp)

    def commit(self):
        jg_commit(self.h)

    def step(self, n_steps: int = 1):
        """Commit pending host-side changes, then queue n_steps steps."""
        jg_commit(self.h)
        jg_step_batch(self.h, n_steps)

    def device_views(self):
        """The device state as torch tensors (zero copy): x (3, stride), q (4, stride), v, w
        (3, stride), in internal body order, and the internal slot of every body."""
        import torch

        jg_commit(self.h)
        (px, pq, pv, pw), stride = jg_device_views(self.h)
        dev = torch.device("cuda", int(self.params.device))

        class _View:
            def __init__(self, ptr, rows):
                self.__cuda_array_interface__ = {"shape": (rows, stride), "typestr": "<f4", "data": (ptr, False),
                                                  "version": 2, "strides": None}

        views = {k: torch.as_tensor(_View(p, r), device=dev)
                 for k, p, r in (("x", px, 3), ("q", pq, 4), ("v", pv, 3), ("w", pw, 3))}
        return views, jg_body_slots(self.h, 0, self.n_bodies)

    def begin_episodes(self):
        """Commit pending changes and start an episode in every tower (jg_begin_episodes)."""
        jg_commit(self.h)
        jg_begin_episodes(self.h)

    def episode(self, tower: int) -> jg_episode:
        return jg_query_episode(self.h, tower)

    def state(self):
        return jg_query_state(self.h, 0, self.n_bodies)

    def set_state(self, pos=None, quat=None, linvel=None, angvel=None):
        jg_set_state(self.h, 0, pos, quat, linvel, angvel)

    def active(self):
        return jg_query_active(self.h, 0, self.n_bodies)

    def contacts(self, tower: int) -> np.ndarray:
        return jg_query_contacts(self.h, tower)

    def stats(self, tower: int = -1) -> jg_stats:
        return jg_query_stats(self.h, tower)

    def features(self, tower: int = -1) -> np.ndarray:
        return jg_query_features(self.h, tower)

    def sync(self):
        jg_sync(self.h)

    def close(self):
        if getattr(self, "h", None) is not None:
            jg_destroy_world(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
