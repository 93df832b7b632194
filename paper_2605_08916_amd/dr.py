"""ctypes binding of libdr.so (include/dr.h), argument marshalling only.

Every function of the C ABI is exposed under the same name; each raises
DrError when the library returns a status other than DR_OK.  The `Scene` and
`Chains` classes wrap the handles for Python callers: they marshal numpy
arrays (host) and torch CUDA tensors (device memory, streams) into the C
calls; all chain-step work runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdr.so")

DR_OK, DR_ERR_INVALID_ARG, DR_ERR_OUT_OF_MEMORY, DR_ERR_DEVICE, DR_ERR_BAD_STATE, DR_ERR_UNSUPPORTED = range(6)
DR_MODE_FUSED, DR_MODE_PLAIN = 0, 1
NO_VERTEX = 0xFFFFFFFF

EXPORTED = [
    "dr_last_error", "dr_version", "dr_bvh_build", "dr_scene_create", "dr_scene_set_camera", "dr_scene_get_stats", "dr_set_allocator",
    "dr_scene_destroy",
    "dr_chains_init", "dr_chains_reinit", "dr_step", "dr_resolve", "dr_image_read", "dr_chains_destroy",
    "dr_chains_read_state", "dr_chains_write_state", "dr_chains_set_record", "dr_chains_set_counters", "dr_stats",
    "dr_chains_set_launch", "dr_chains_get_launch", "dr_eval_logp_grad", "dr_eval_logp_grad_noalloc", "dr_pt_render",
    "dr_frame_capture", "dr_frame_launch", "dr_frame_destroy", "dr_mixture_run", "dr_mixture_step",
]


class DrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"dr status {status}: {msg}")
        self.status = status


# ---------------------------------------------------------------------------
# C structures (mirror include/dr.h)
# ---------------------------------------------------------------------------
class dr_quad_light(C.Structure):
    _fields_ = [("p0", C.c_float * 3), ("e1", C.c_float * 3), ("e2", C.c_float * 3), ("Le", C.c_float * 3)]


class dr_material(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("albedo", C.c_float * 3), ("roughness", C.c_float), ("f0", C.c_float * 3),
                ("Le", C.c_float * 3), ("eta", C.c_float)]


DR_MAT_LAMBERT, DR_MAT_GGX_CONDUCTOR, DR_MAT_SMOOTH_CONDUCTOR, DR_MAT_SMOOTH_DIELECTRIC = 0, 1, 2, 3


class dr_bvh_node(C.Structure):
    _fields_ = [("lo", C.c_float * 3), ("hi", C.c_float * 3), ("a", C.c_int32), ("b", C.c_int32)]


class dr_camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("at", C.c_float * 3), ("up", C.c_float * 3), ("vfov_deg", C.c_float),
                ("width", C.c_uint32), ("height", C.c_uint32)]



ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
# Every callback pair ever installed stays referenced for the life of the
# process: buffers allocated through a pair are freed through it later, also
# after another allocator has been installed.
_hooks_alive = []


def use_torch_allocator(enable: bool = True):
    """Serve the library's device buffers from torch's caching allocator (or
    go back to hipMalloc/hipFree).  Buffers keep the allocator that made them."""
    if not enable:
        _check(lib().dr_set_allocator(ALLOC_FN(), FREE_FN(), None))
        return
    import torch

    def _alloc(nbytes, stream, user):
        try:
            s = stream if stream else torch.cuda.current_stream().cuda_stream
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(s))
        except Exception:
            return None

    def _free(ptr, nbytes, stream, user):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass

    hooks = (ALLOC_FN(_alloc), FREE_FN(_free))
    _hooks_alive.append(hooks)
    _check(lib().dr_set_allocator(hooks[0], hooks[1], None))


class dr_scene_stats(C.Structure):
    _fields_ = [("n_triangles", C.c_uint32), ("n_nodes", C.c_uint32), ("stack_entries", C.c_uint32),
                ("stack_bytes_per_lane", C.c_uint32)]


class dr_scene_desc(C.Structure):
    _fields_ = [("vertices", C.POINTER(C.c_float)), ("n_vertices", C.c_uint32),
                ("indices", C.POINTER(C.c_uint32)), ("n_triangles", C.c_uint32),
                ("tri_material", C.POINTER(C.c_uint32)), ("materials", C.POINTER(dr_material)),
                ("n_materials", C.c_uint32), ("lights", C.POINTER(dr_quad_light)), ("n_lights", C.c_uint32),
                ("bvh", C.POINTER(dr_bvh_node)), ("n_nodes", C.c_uint32), ("bvh_prim_order", C.POINTER(C.c_uint32)),
                ("camera", dr_camera)]


class dr_params(C.Structure):
    _fields_ = [("n_chains", C.c_uint32), ("max_path_len", C.c_uint32), ("stddev", C.c_float), ("dt", C.c_float),
                ("gamma", C.c_float), ("m", C.c_float), ("eps", C.c_float), ("k0", C.c_float),
                ("rao_blackwell", C.c_uint32), ("mode", C.c_uint32), ("sigma_diag", C.c_void_p)]


class dr_state(C.Structure):
    _fields_ = [("x", C.POINTER(C.c_float)), ("score", C.POINTER(C.c_float)), ("killed", C.POINTER(C.c_uint32)),
                ("accum", C.POINTER(C.c_float)), ("p", C.POINTER(C.c_float)), ("weight", C.POINTER(C.c_float)),
                ("pixel", C.POINTER(C.c_uint32)), ("f_over_p", C.POINTER(C.c_float)),
                ("path_rec", C.POINTER(C.c_uint32)), ("step", C.c_uint64), ("tour_count", C.c_uint64),
                ("k0", C.c_double), ("p_lambda_hat", C.c_double)]


class dr_mixture_desc(C.Structure):
    _fields_ = [("d", C.c_uint32), ("n_modes", C.c_uint32), ("weights", C.POINTER(C.c_float)),
                ("means", C.POINTER(C.c_float)), ("stds", C.POINTER(C.c_float)), ("c0", C.c_float)]


class dr_counters(C.Structure):
    _fields_ = [("chain_steps", C.c_uint64), ("rays", C.c_uint64), ("node_visits", C.c_uint64),
                ("tri_tests", C.c_uint64), ("kills", C.c_uint64), ("tours", C.c_uint64), ("adjoints", C.c_uint64),
                ("k0", C.c_double), ("p_lambda_hat", C.c_double)]


class dr_launch_cfg(C.Structure):
    _fields_ = [("block", C.c_uint32), ("blocks_per_cu", C.c_uint32), ("grab", C.c_uint32),
                ("lanes_per_chain", C.c_uint32), ("sort_by_length", C.c_uint32), ("refill", C.c_uint32),
                ("refill_event_pct", C.c_uint32), ("refill_advance_pct", C.c_uint32), ("sort_by_tile", C.c_uint32),
                ("wavefront", C.c_uint32), ("init_refill", C.c_uint32)]


_lib = None


def lib():
    """Load libdr.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    pp = C.POINTER(C.c_void_p)
    st = C.c_int
    sig = {
        "dr_last_error": ([], C.c_char_p),
        "dr_version": ([], C.c_char_p),
        "dr_bvh_build": ([C.POINTER(C.c_float), C.c_uint32, C.POINTER(C.c_uint32), C.c_uint32, C.c_uint32,
                          C.POINTER(dr_bvh_node), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)], st),
        "dr_scene_create": ([C.POINTER(dr_scene_desc), C.c_int, pp], st),
        "dr_scene_set_camera": ([P, C.POINTER(dr_camera)], st),
        "dr_scene_destroy": ([P], None),
        "dr_scene_get_stats": ([P, C.POINTER(dr_scene_stats)], st),
        "dr_set_allocator": ([ALLOC_FN, FREE_FN, P], st),
        "dr_chains_init": ([P, C.POINTER(dr_params), C.c_uint64, C.c_uint32, P, pp], st),
        "dr_chains_reinit": ([P, C.c_uint32, P], st),
        "dr_step": ([P, C.c_uint32, P], st),
        "dr_resolve": ([P, P, P], st),
        "dr_image_read": ([P, C.POINTER(C.c_float), C.POINTER(C.c_uint64), P], st),
        "dr_chains_destroy": ([P], st),
        "dr_chains_read_state": ([P, C.POINTER(dr_state), P], st),
        "dr_chains_write_state": ([P, C.POINTER(dr_state), P], st),
        "dr_chains_set_record": ([P, C.c_int], st),
        "dr_chains_set_counters": ([P, C.c_int], st),
        "dr_stats": ([P, C.POINTER(dr_counters), P], st),
        "dr_chains_set_launch": ([P, C.POINTER(dr_launch_cfg)], st),
        "dr_chains_get_launch": ([P, C.POINTER(dr_launch_cfg)], st),
        "dr_eval_logp_grad": ([P, C.c_uint32, P, C.c_uint32, C.c_float, P, P, P, P, P], st),
        "dr_eval_logp_grad_noalloc": ([P, C.c_uint32, P, C.c_uint32, C.c_float, P, P, P, P, P], st),
        "dr_pt_render": ([P, C.c_uint32, C.c_uint64, C.c_uint32, P, P], st),
        "dr_frame_capture": ([P, C.c_uint32, C.c_int, P, P, pp], st),
        "dr_frame_launch": ([P, P], st),
        "dr_frame_destroy": ([P], st),
        "dr_mixture_run": ([C.POINTER(dr_mixture_desc), C.POINTER(dr_params), C.c_uint64, C.c_uint32, C.c_uint32,
                            C.c_uint32, C.POINTER(C.c_double), C.POINTER(C.c_uint64), C.POINTER(C.c_double),
                            C.POINTER(C.c_double), P], st),
        "dr_mixture_step": ([C.POINTER(dr_mixture_desc), C.POINTER(dr_params), C.c_uint64, C.c_uint64, C.c_double,
                             C.POINTER(C.c_float), C.POINTER(C.c_float), C.POINTER(C.c_uint32), C.POINTER(C.c_float),
                             C.POINTER(C.c_float), P], st),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(status):
    if status != DR_OK:
        raise DrError(status, lib().dr_last_error().decode())


def _fp(a, ct=C.c_float):
    return None if a is None else a.ctypes.data_as(C.POINTER(ct))


def _stream(stream=None):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# Same-name wrappers of the C entry points
# ---------------------------------------------------------------------------
def dr_version() -> str:
    return lib().dr_version().decode()


def dr_bvh_build(vertices: np.ndarray, indices: np.ndarray, max_leaf: int = 2):
    V = np.ascontiguousarray(vertices, np.float32).reshape(-1, 3)
    I = np.ascontiguousarray(indices, np.uint32).reshape(-1, 3)
    T = I.shape[0]
    nodes = (dr_bvh_node * max(1, 2 * T))()
    order = np.zeros(T, np.uint32)
    nn = C.c_uint32(0)
    _check(lib().dr_bvh_build(_fp(V), V.shape[0], _fp(I, C.c_uint32), T, max_leaf, nodes, C.byref(nn),
                              _fp(order, C.c_uint32)))
    arr = np.ctypeslib.as_array(nodes)[: nn.value].copy()
    return arr, order


def _camera(cam: np.ndarray, W: int, H: int) -> dr_camera:
    c = dr_camera()
    c.eye[:] = [float(v) for v in cam[0:3]]
    c.at[:] = [float(v) for v in cam[3:6]]
    c.up[:] = [float(v) for v in cam[6:9]]
    c.vfov_deg = float(cam[9])
    c.width, c.height = int(W), int(H)
    return c


def dr_scene_create(sc: dict, device: int = 0, bvh=None):
    """Create a device scene from a scene dict (see inputs.py).  bvh =
    (nodes, prim_order) from dr_bvh_build, or None to let the library build."""
    V = np.ascontiguousarray(sc["vertices"], np.float32)
    I = np.ascontiguousarray(sc["indices"], np.uint32)
    TM = np.ascontiguousarray(sc["tri_material"], np.uint32)
    M = np.asarray(sc["materials"], np.float32)
    Lt = np.asarray(sc["lights"], np.float32)
    mats = (dr_material * M.shape[0])()
    for i, q in enumerate(M):
        mats[i].kind = int(q[0])
        mats[i].albedo[:] = [float(v) for v in q[1:4]]
        mats[i].roughness = float(q[4])
        mats[i].f0[:] = [float(v) for v in q[5:8]]
        mats[i].Le[:] = [float(v) for v in q[8:11]]
        mats[i].eta = float(q[11]) if q.shape[0] > 11 else 1.0
    lights = (dr_quad_light * Lt.shape[0])()
    for i, q in enumerate(Lt):
        lights[i].p0[:] = [float(v) for v in q[0:3]]
        lights[i].e1[:] = [float(v) for v in q[3:6]]
        lights[i].e2[:] = [float(v) for v in q[6:9]]
        lights[i].Le[:] = [float(v) for v in q[9:12]]
    desc = dr_scene_desc()
    desc.vertices, desc.n_vertices = _fp(V), V.shape[0]
    desc.indices, desc.n_triangles = _fp(I, C.c_uint32), I.shape[0]
    desc.tri_material = _fp(TM, C.c_uint32)
    desc.materials, desc.n_materials = C.cast(mats, C.POINTER(dr_material)), M.shape[0]
    desc.lights, desc.n_lights = C.cast(lights, C.POINTER(dr_quad_light)), Lt.shape[0]
    keep = [V, I, TM, mats, lights]
    if bvh is not None:
        nodes, order = bvh
        nodes = np.ascontiguousarray(nodes)
        order = np.ascontiguousarray(order, np.uint32)
        keep += [nodes, order]
        desc.bvh = nodes.ctypes.data_as(C.POINTER(dr_bvh_node))
        desc.n_nodes = nodes.shape[0]
        desc.bvh_prim_order = _fp(order, C.c_uint32)
    desc.camera = _camera(sc["camera"], sc["width"], sc["height"])
    h = C.c_void_p()
    _check(lib().dr_scene_create(C.byref(desc), device, C.byref(h)))
    del keep
    return h


class Scene:
    def __init__(self, sc: dict, device: int = 0, bvh=None, max_leaf: int = 2):
        if bvh is None:
            bvh = dr_bvh_build(sc["vertices"], sc["indices"], max_leaf)
        self.sc = sc
        self.W, self.H = int(sc["width"]), int(sc["height"])
        self.h = dr_scene_create(sc, device, bvh)

    def set_camera(self, cam):
        c = _camera(np.asarray(cam, np.float32), self.W, self.H)
        _check(lib().dr_scene_set_camera(self.h, C.byref(c)))

    def stats(self) -> dict:
        o = dr_scene_stats()
        _check(lib().dr_scene_get_stats(self.h, C.byref(o)))
        return {k: getattr(o, k) for k, _ in dr_scene_stats._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib().dr_scene_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def eval_logp_grad(self, L: int, u, eps: float = 1e-8, grad: bool = True, rec: bool = False, stream=None):
        """u: CUDA float32 tensor (n, d).  Returns (f, logp, grad or None,
        rec or None) as CUDA tensors."""
        import torch
        u = u.contiguous()
        n = u.shape[0]
        d = 4 * (L - 1)
        assert u.dtype == torch.float32 and u.is_cuda and u.shape[1] == d
        f = torch.empty((n, 3), device=u.device, dtype=torch.float32)
        logp = torch.empty((n,), device=u.device, dtype=torch.float32)
        g = torch.empty((n, d), device=u.device, dtype=torch.float32) if grad else None
        r = torch.empty((n, L - 1), device=u.device, dtype=torch.int32) if rec else None
        _check(lib().dr_eval_logp_grad(self.h, L, _dev_ptr(u), n, eps, _dev_ptr(f), _dev_ptr(logp), _dev_ptr(g),
                                       _dev_ptr(r), _stream(stream)))
        return f, logp, g, r

    def eval_logp_grad_into(self, L: int, u, f, logp, grad=None, rec=None, eps: float = 1e-8, stream=None):
        """dr_eval_logp_grad_noalloc: the same evaluation into caller-owned
        CUDA tensors (f (n, 3), logp (n,), grad (n, d) or None, rec (n, L-1)
        int32 or None), with the library's fixed scratch buffer."""
        import torch
        n = u.shape[0]
        assert u.dtype == torch.float32 and u.is_cuda and u.is_contiguous() and u.shape[1] == 4 * (L - 1)
        for t, shape in ((f, (n, 3)), (logp, (n,)), (grad, (n, 4 * (L - 1))), (rec, (n, L - 1))):
            assert t is None or (t.is_cuda and t.is_contiguous() and tuple(t.shape) == shape)
        _check(lib().dr_eval_logp_grad_noalloc(self.h, L, _dev_ptr(u), n, eps, _dev_ptr(f), _dev_ptr(logp),
                                               _dev_ptr(grad), _dev_ptr(rec), _stream(stream)))

    def pt_render(self, L: int, seed: int, spp: int, stream=None):
        import torch
        img = torch.empty((3, self.H * self.W), device="cuda", dtype=torch.float32)
        _check(lib().dr_pt_render(self.h, L, seed, spp, _dev_ptr(img), _stream(stream)))
        return img


def make_params(n_chains: int, L: int, stddev=5e-3, dt=1e-5, gamma=0.5, m=64.0, eps=1e-8, k0=0.0,
                rao_blackwell=1, mode=DR_MODE_FUSED, sigma=None) -> dr_params:
    p = dr_params()
    p.n_chains, p.max_path_len = n_chains, L
    p.stddev, p.dt, p.gamma, p.m, p.eps, p.k0 = stddev, dt, gamma, m, eps, k0
    p.rao_blackwell, p.mode = rao_blackwell, mode
    p.sigma_diag = None if sigma is None else sigma.data_ptr()
    return p


class Chains:
    """Chain ensemble on a device scene (dr_chains_init ... dr_chains_destroy)."""

    def __init__(self, scene: Scene, n_chains: int, L: int, seed: int, frame: int = 0, sigma=None, stream=None,
                 record: bool = False, **kw):
        self.scene = scene
        self.N, self.L, self.d = n_chains, L, 4 * (L - 1)
        self.sigma = sigma  # keep the borrowed device buffer alive
        self.params = make_params(n_chains, L, sigma=sigma, **kw)
        self.h = C.c_void_p()
        self._init_args = (seed, frame)
        h = C.c_void_p()
        # recording must be on before the init pass to capture it
        _check(lib().dr_chains_init(scene.h, C.byref(self.params), seed, frame, _stream(stream), C.byref(h)))
        self.h = h
        if record:
            self.set_record(True)

    def close(self):
        if getattr(self, "h", None):
            lib().dr_chains_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reinit(self, frame: int, stream=None):
        _check(lib().dr_chains_reinit(self.h, frame, _stream(stream)))

    def step(self, n: int = 1, stream=None):
        _check(lib().dr_step(self.h, n, _stream(stream)))

    def resolve(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((3, self.scene.H * self.scene.W), device="cuda", dtype=torch.float32)
        _check(lib().dr_resolve(self.h, _dev_ptr(out), _stream(stream)))
        return out

    def image_read(self, stream=None):
        img = np.zeros((3, self.scene.H * self.scene.W), np.float32)
        tours = C.c_uint64(0)
        _check(lib().dr_image_read(self.h, _fp(img), C.byref(tours), _stream(stream)))
        return img, tours.value

    def set_record(self, on: bool):
        _check(lib().dr_chains_set_record(self.h, 1 if on else 0))

    def set_counters(self, on: bool):
        _check(lib().dr_chains_set_counters(self.h, 1 if on else 0))

    def stats(self, stream=None) -> dict:
        c = dr_counters()
        _check(lib().dr_stats(self.h, C.byref(c), _stream(stream)))
        return {k: getattr(c, k) for k, _ in dr_counters._fields_}

    def set_launch(self, block=0, blocks_per_cu=0, grab=0, lanes_per_chain=0, sort_by_length=0, refill=0,
                   refill_event_pct=0, refill_advance_pct=0, sort_by_tile=0, wavefront=0,
                   init_refill=0):
        """Zero keeps a field; sort_by_length, refill, sort_by_tile, wavefront and init_refill: 1 on, 2 off."""
        cfg = dr_launch_cfg(block, blocks_per_cu, grab, lanes_per_chain, sort_by_length, refill, refill_event_pct,
                            refill_advance_pct, sort_by_tile, wavefront, init_refill)
        _check(lib().dr_chains_set_launch(self.h, C.byref(cfg)))

    def get_launch(self) -> dict:
        cfg = dr_launch_cfg()
        _check(lib().dr_chains_get_launch(self.h, C.byref(cfg)))
        return {k: getattr(cfg, k) for k, _ in dr_launch_cfg._fields_}

    def read_state(self, stream=None) -> dict:
        N, d, V = self.N, self.d, self.L - 1
        npx = self.scene.W * self.scene.H
        out = dict(x=np.zeros((d, N), np.float32), score=np.zeros((d, N), np.float32),
                   killed=np.zeros(N, np.uint32), accum=np.zeros((3, npx), np.float32), p=np.zeros(N, np.float32),
                   weight=np.zeros(N, np.float32), pixel=np.zeros(N, np.uint32),
                   f_over_p=np.zeros((3, N), np.float32), path_rec=np.zeros((V, N), np.uint32))
        s = dr_state()
        s.x, s.score, s.killed, s.accum = _fp(out["x"]), _fp(out["score"]), _fp(out["killed"], C.c_uint32), _fp(out["accum"])
        s.p, s.weight, s.pixel = _fp(out["p"]), _fp(out["weight"]), _fp(out["pixel"], C.c_uint32)
        s.f_over_p, s.path_rec = _fp(out["f_over_p"]), _fp(out["path_rec"], C.c_uint32)
        _check(lib().dr_chains_read_state(self.h, C.byref(s), _stream(stream)))
        out.update(step=s.step, tour_count=s.tour_count, k0=s.k0, p_lambda_hat=s.p_lambda_hat)
        return out

    def capture_frame(self, n_steps: int, reinit: bool, image, stream) -> "Frame":
        """Capture re-init (optional) + n_steps + resolve into `image` (CUDA
        float32 (3, W*H)) as a HIP graph on `stream` (a torch.cuda.Stream)."""
        h = C.c_void_p()
        _check(lib().dr_frame_capture(self.h, n_steps, 1 if reinit else 0, _dev_ptr(image),
                                      C.c_void_p(stream.cuda_stream), C.byref(h)))
        return Frame(h, self, image)

    def write_state(self, x=None, score=None, killed=None, accum=None, step=None, tour_count=0, k0=0.0, stream=None):
        s = dr_state()
        keep = []
        for name, arr, ct, dt in (("x", x, C.c_float, np.float32), ("score", score, C.c_float, np.float32),
                                  ("killed", killed, C.c_uint32, np.uint32), ("accum", accum, C.c_float, np.float32)):
            if arr is not None:
                a = np.ascontiguousarray(arr, dt)
                keep.append(a)
                setattr(s, name, _fp(a, ct))
        s.step = self.read_state()["step"] if step is None else step
        s.tour_count = tour_count
        s.k0 = k0
        _check(lib().dr_chains_write_state(self.h, C.byref(s), _stream(stream)))


class Frame:
    """A captured frame (dr_frame_capture / dr_frame_launch / dr_frame_destroy)."""

    def __init__(self, h, chains, image):
        self.h, self.chains, self.image = h, chains, image

    def launch(self, stream):
        _check(lib().dr_frame_launch(self.h, C.c_void_p(stream.cuda_stream)))

    def close(self):
        if getattr(self, "h", None):
            lib().dr_frame_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mixture:
    """Analytic target of the chain step (dr_mixture_run / dr_mixture_step):
    a wrapped Gaussian mixture on T^d with floor c0; f = p g with the test
    functions (1, cos 2 pi x_i, sin 2 pi x_i)."""

    def __init__(self, d: int, weights, means, stds, c0: float):
        self.d = int(d)
        self.w = np.ascontiguousarray(weights, np.float32).reshape(-1)
        self.m = np.ascontiguousarray(means, np.float32).reshape(-1, self.d) if self.w.size else np.zeros((0, self.d),
                                                                                                          np.float32)
        self.s = np.ascontiguousarray(stds, np.float32).reshape(-1)
        self.desc = dr_mixture_desc(self.d, self.w.size, _fp(self.w), _fp(self.m), _fp(self.s), float(c0))

    def run(self, n_chains: int, seed: int, n_steps: int, n_batches: int = 32, frame: int = 0, sigma=None,
            stream=None, **kw) -> dict:
        """Initialise + n_steps steps; returns per-batch accumulators (units of
        dt), tours, k0, p_lambda and the estimate k0 dt accum / tours."""
        p = make_params(n_chains, 2, sigma=sigma, **kw)
        nf = 1 + 2 * self.d
        acc = np.zeros((n_batches, nf))
        tours = np.zeros(n_batches, np.uint64)
        k0, pl = C.c_double(0), C.c_double(0)
        _check(lib().dr_mixture_run(C.byref(self.desc), C.byref(p), seed, frame, n_steps, n_batches,
                                    _fp(acc, C.c_double), _fp(tours, C.c_uint64), C.byref(k0), C.byref(pl),
                                    _stream(stream)))
        est = k0.value * p.dt * acc.sum(0) / max(1, int(tours.sum()))
        return dict(batch_accum=acc, batch_tours=tours, k0=k0.value, p_lambda=pl.value, estimate=est, dt=p.dt)

    def step(self, x, score, killed, seed: int, step: int, k0: float, sigma=None, stream=None, **kw) -> dict:
        """One evolve step from a host state (x, score: d x N; killed: N)."""
        x = np.array(x, np.float32, order="C", copy=True)
        score = np.array(score, np.float32, order="C", copy=True)
        killed = np.array(killed, np.uint32, order="C", copy=True)
        n = killed.shape[0]
        assert x.shape == (self.d, n) and score.shape == (self.d, n)
        p = make_params(n, 2, sigma=sigma, **kw)
        pv = np.zeros(n, np.float32)
        wv = np.zeros(n, np.float32)
        _check(lib().dr_mixture_step(C.byref(self.desc), C.byref(p), seed, step, k0, _fp(x), _fp(score),
                                     _fp(killed, C.c_uint32), _fp(pv), _fp(wv), _stream(stream)))
        return dict(x=x, score=score, killed=killed, p=pv, w=wv)
