"""Scene: a batch of environments stepped by libnsn on one GPU."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


def params_c(p) -> L.ParamsC:
    """C parameter struct from any object with the SolverParams fields."""
    return L.ParamsC(ncp=int(p.ncp), rmode=int(p.rmode), damping=float(p.damping), eps=float(p.eps),
                     geo_stiff=int(p.geo_stiff), fem_mode=int(p.fem_mode), margin=float(p.margin),
                     warm=int(p.warm), line_search=int(getattr(p, "line_search", 0)),
                     linear=int(getattr(p, "linear", 0)), islands=int(getattr(p, "islands", 0)),
                     watchdog=int(getattr(p, "watchdog", 0)))


def stats_to_dicts(arr):
    return [{k: arr[k][i].item() for k in arr.dtype.names} for i in range(len(arr))]


class _Marshal:
    """Keeps the float32/int32 copies of the descriptors alive during create."""

    def __init__(self, envs):
        self.keep = []
        self.c = (L.EnvDescC * len(envs))()
        for i, d in enumerate(envs):
            s = self.c[i]
            s.n_rigid = d.n_rigid
            s.n_particles = d.n_particles
            s.n_tets = d.n_tets
            s.n_joints = d.n_joints
            for name in ["rigid_mass", "rigid_inertia", "rigid_x", "rigid_q", "rigid_v", "rigid_w",
                         "rigid_extent", "particle_x", "particle_v", "particle_rest", "particle_mass",
                         "tet_material", "joint_anchor", "joint_axis", "joint_ref", "joint_drive"]:
                a = np.ascontiguousarray(getattr(d, name), dtype=np.float32).ravel()
                if a.size == 0:
                    a = np.zeros(1, np.float32)
                self.keep.append(a)
                setattr(s, name, L.fptr(a))
            for name in ["rigid_shape", "tet_ids", "joint_type", "joint_body"]:
                a = np.ascontiguousarray(getattr(d, name), dtype=np.int32).ravel()
                if a.size == 0:
                    a = np.zeros(1, np.int32)
                self.keep.append(a)
                setattr(s, name, L.iptr(a))
            s.mu = float(d.mu)
            s.gravity = (C.c_float * 3)(*d.gravity)
            s.ground = int(d.ground)
            s.max_contacts = int(d.max_contacts)
            s.tet_model = int(getattr(d, "tet_model", 0))


class Scene:
    """A batch of environments on one GPU.

    envs: list of scene_inputs.EnvDesc; params: object with the SolverParams fields.
    The device workspace is one torch uint8 tensor.  The scene runs on its own stream
    (default priority) unless `stream` is given: steps are then captured once and
    replayed from a hipGraph, and the launch buckets of a step run on streams forked
    from it (the library launches directly, in order, on the null stream).  Calls that
    return data synchronise that stream; torch work that reads scene memory must wait
    for it.  reserve: extra parameter objects whose options (islands, line search) the
    workspace must also hold, for later set_params calls."""

    def __init__(self, envs, params, device="cuda", stream=None, reserve=()):
        import torch

        self.torch = torch
        self.lib = L.lib()
        self.envs = list(envs)
        self.n_envs = len(self.envs)
        m = _Marshal(self.envs)
        nbytes = C.c_size_t(0)
        pc = params_c(params)
        for r in reserve:  # the union of the options the scene may use
            rc = params_c(r)
            pc.islands = max(pc.islands, rc.islands)
            pc.line_search = max(pc.line_search, rc.line_search)
        self._reserved = pc
        L.check(self.lib.nsn_query_workspace(m.c, self.n_envs, C.byref(pc), C.byref(nbytes)),
                "nsn_query_workspace")
        self.workspace_bytes = int(nbytes.value)
        self.device = torch.device(device)
        self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.workspace.record_stream(self.stream)
        self._params = params
        h = C.c_void_p()
        L.check(self.lib.nsn_create_scene(m.c, self.n_envs, C.byref(pc), C.c_void_p(self.stream.cuda_stream),
                                          C.c_void_p(self.workspace.data_ptr()), self.workspace_bytes,
                                          C.byref(h)), "nsn_create_scene")
        self.h = h
        self.use_graphs = self.stream.cuda_stream != 0
        if (pc.islands, pc.line_search) != (params_c(params).islands, params_c(params).line_search):
            self.set_params(params)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.nsn_destroy_scene(h)
            self.h = None

    # ---- stepping ----
    def set_params(self, params):
        pc = params_c(params)
        L.check(self.lib.nsn_set_params(self.h, C.byref(pc)), "nsn_set_params")
        self._params = params

    def step(self, h, newton_iters, cr_iters, tol=0.0, with_stats=False):
        """One time step (asynchronous); with_stats: synchronise and return the stats."""
        out = np.zeros(self.n_envs, L.STATS_DTYPE) if with_stats else None
        L.check(self.lib.nsn_step(self.h, float(h), int(newton_iters), int(cr_iters), float(tol),
                                  out.ctypes.data if out is not None else None), "nsn_step")
        return out

    # ---- parity hooks ----
    def set_contacts(self, env, key, bodies, normal, a_local, b_local, thickness):
        """Replace collision detection of `env` for the next step by this contact list
        (keys ascending, feature bodies non-decreasing)."""
        n = len(key)
        arr = (L.ContactC * max(n, 1))()
        for i in range(n):
            c = arr[i]
            c.key = int(key[i])
            c.body_a, c.body_b = int(bodies[i][0]), int(bodies[i][1])
            c.normal = (C.c_float * 3)(*[float(v) for v in normal[i]])
            c.a_local = (C.c_float * 3)(*[float(v) for v in a_local[i]])
            c.b_local = (C.c_float * 3)(*[float(v) for v in b_local[i]])
            c.thickness = float(thickness[i])
        L.check(self.lib.nsn_set_contacts(self.h, int(env), arr, n), "nsn_set_contacts")

    def dump_iteration(self, h, k, cr_iters):
        """A step of every env that stops inside Newton iteration k (see nsn.h)."""
        L.check(self.lib.nsn_dump_iteration(self.h, float(h), int(k), int(cr_iters)), "nsn_dump_iteration")
        self._dumped_k = int(k)

    def read_iteration(self, env, fields=None):
        """{field: float32 array} of the last dump step for one env (nsn_read_iteration)."""
        out = {}
        names = fields or [f for f in L.IT_FIELDS if getattr(self, "_dumped_k", 0) >= 1 or not f.startswith("prev_")]
        for name in names:
            fi = L.IT_FIELDS.index(name)
            n = C.c_int32(0)
            L.check(self.lib.nsn_read_iteration(self.h, int(env), fi, 0, C.byref(n), None), "nsn_read_iteration")
            a = np.zeros(max(n.value, 1), np.float32)
            L.check(self.lib.nsn_read_iteration(self.h, int(env), fi, n.value, C.byref(n), L.fptr(a)),
                    "nsn_read_iteration")
            out[name] = a[:n.value]
        return out

    def stats(self):
        out = np.zeros(self.n_envs, L.STATS_DTYPE)
        L.check(self.lib.nsn_get_stats(self.h, out.ctypes.data), "nsn_get_stats")
        return out

    def synchronize(self):
        self.stream.synchronize()

    # ---- state I/O ----
    def read_state(self, env):
        d = self.envs[env]
        rx = np.zeros((d.n_rigid, 3), np.float32); rq = np.zeros((d.n_rigid, 4), np.float32)
        rv = np.zeros((d.n_rigid, 3), np.float32); rw = np.zeros((d.n_rigid, 3), np.float32)
        px = np.zeros((d.n_particles, 3), np.float32); pv = np.zeros((d.n_particles, 3), np.float32)
        t = C.c_double(0.0)
        L.check(self.lib.nsn_read_state(self.h, env, L.fptr(rx), L.fptr(rq), L.fptr(rv), L.fptr(rw),
                                        L.fptr(px), L.fptr(pv), C.byref(t)), "nsn_read_state")
        return dict(rigid_x=rx, rigid_q=rq, rigid_v=rv, rigid_w=rw, particle_x=px, particle_v=pv,
                    time=t.value)

    def save_state(self):
        """Snapshot of every env's dynamic state (nsn_save_state) in a device buffer."""
        import torch

        n = C.c_size_t(0)
        L.check(self.lib.nsn_state_bytes(self.h, C.byref(n)), "nsn_state_bytes")
        buf = torch.empty(int(n.value), dtype=torch.uint8, device=self.device)
        buf.record_stream(self.stream)
        L.check(self.lib.nsn_save_state(self.h, C.c_void_p(buf.data_ptr())), "nsn_save_state")
        return buf

    def load_state(self, buf):
        """Restore a snapshot taken by save_state of this scene (nsn_load_state)."""
        L.check(self.lib.nsn_load_state(self.h, C.c_void_p(buf.data_ptr())), "nsn_load_state")

    def write_state(self, env, st):
        d = self.envs[env]

        def g(k, shape):
            if k not in st or st[k] is None:
                return None
            return L.f32(np.asarray(st[k]).reshape(shape))
        arrs = [g("rigid_x", (d.n_rigid, 3)), g("rigid_q", (d.n_rigid, 4)), g("rigid_v", (d.n_rigid, 3)),
                g("rigid_w", (d.n_rigid, 3)), g("particle_x", (d.n_particles, 3)),
                g("particle_v", (d.n_particles, 3))]
        t = C.c_double(st["time"]) if "time" in st and st["time"] is not None else None
        L.check(self.lib.nsn_write_state(self.h, env, *[L.fptr(a) for a in arrs],
                                         C.byref(t) if t is not None else None), "nsn_write_state")

    def contacts(self, env):
        cap = self.envs[env].max_contacts
        n = C.c_int32(0)
        keys = np.zeros(max(cap, 1), np.int32); bodies = np.zeros((max(cap, 1), 2), np.int32)
        geom = np.zeros((max(cap, 1), 10), np.float32); lam = np.zeros((max(cap, 1), 3), np.float32)
        L.check(self.lib.nsn_read_contacts(self.h, env, cap, C.byref(n), L.iptr(keys), L.iptr(bodies),
                                           L.fptr(geom), L.fptr(lam)), "nsn_read_contacts")
        k = min(n.value, cap)
        return dict(key=keys[:k].astype(np.int64), bodies=bodies[:k], normal=geom[:k, 0:3],
                    a_local=geom[:k, 3:6], b_local=geom[:k, 6:9], thickness=geom[:k, 9], lam=lam[:k])

    def lambdas(self, env):
        d = self.envs[env]
        cap = 6 * d.n_joints + (6 if getattr(d, "tet_model", 0) == 1 else 3) * d.n_tets + 3 * d.max_contacts
        out = np.zeros(max(cap, 1), np.float32)
        n = C.c_int32(0)
        L.check(self.lib.nsn_read_lambda(self.h, env, cap, C.byref(n), L.fptr(out)), "nsn_read_lambda")
        return out[:n.value]

    def enable_features(self, on=True):
        L.check(self.lib.nsn_enable_features(self.h, int(bool(on))), "nsn_enable_features")

    def features(self, env):
        cap = self.envs[env].max_contacts
        out = np.zeros((max(cap, 1), 12), np.float32)
        n = C.c_int32(0)
        L.check(self.lib.nsn_read_features(self.h, env, cap, C.byref(n), L.fptr(out)), "nsn_read_features")
        return out[:min(n.value, cap)]

    def set_warm_start_model(self, blob):
        b = L.f32(blob).ravel()
        L.check(self.lib.nsn_set_warm_start_model(self.h, L.fptr(b), b.size), "nsn_set_warm_start_model")

    def set_use_graphs(self, on):
        L.check(self.lib.nsn_set_use_graphs(self.h, int(bool(on))), "nsn_set_use_graphs")
        self.use_graphs = bool(on) and self.stream.cuda_stream != 0

    use_graphs = True  # the library's default for a scene with its own stream

    def accumulators(self):
        out = np.zeros(self.n_envs, L.ACC_DTYPE)
        L.check(self.lib.nsn_read_accumulators(self.h, out.ctypes.data), "nsn_read_accumulators")
        return out

    def reset_accumulators(self):
        L.check(self.lib.nsn_reset_accumulators(self.h), "nsn_reset_accumulators")

    def kernel_times_ms(self, cap=1024):
        out = np.zeros(cap, np.float64)
        n = C.c_int32(0)
        L.check(self.lib.nsn_read_kernel_times(self.h, cap, C.byref(n), out.ctypes.data_as(L.D)),
                "nsn_read_kernel_times")
        return out[:n.value]

    # ---- schedule ----
    def env_order(self):
        out = np.zeros(self.n_envs, np.int32)
        L.check(self.lib.nsn_get_env_order(self.h, L.iptr(out)), "nsn_get_env_order")
        return out

    def set_schedule(self, buckets):
        """buckets: list of (first, count, block) tiling the env order."""
        first = np.array([b[0] for b in buckets], np.int32)
        count = np.array([b[1] for b in buckets], np.int32)
        block = np.array([b[2] for b in buckets], np.int32)
        L.check(self.lib.nsn_set_schedule(self.h, len(buckets), L.iptr(first), L.iptr(count), L.iptr(block)),
                "nsn_set_schedule")

    def set_lds_mode(self, max_mode):
        """0: body-space vector in global memory; 1: in LDS; 2: with the tets'
        contributions in LDS where they fit (default).  Same results."""
        L.check(self.lib.nsn_set_lds_mode(self.h, int(max_mode)), "nsn_set_lds_mode")

    pcr_form = 2  # the library's default

    def set_pcr_form(self, form):
        """0: streaming two-pass PCR; 1: register-resident where an env's elements fit
        (results identical to 0); 2: one-pass (default) (nsn_set_pcr_form)."""
        L.check(self.lib.nsn_set_pcr_form(self.h, int(form)), "nsn_set_pcr_form")
        self.pcr_form = int(form)

    def lds_modes(self):
        """LDS mode of every current bucket."""
        cap = 64
        n = C.c_int32(0)
        m = np.zeros(cap, np.int32)
        L.check(self.lib.nsn_get_lds_modes(self.h, cap, C.byref(n), L.iptr(m)), "nsn_get_lds_modes")
        return [int(v) for v in m[:n.value]]

    def schedule(self):
        cap = 64
        n = C.c_int32(0)
        f, c, b = np.zeros(cap, np.int32), np.zeros(cap, np.int32), np.zeros(cap, np.int32)
        L.check(self.lib.nsn_get_schedule(self.h, cap, C.byref(n), L.iptr(f), L.iptr(c), L.iptr(b)),
                "nsn_get_schedule")
        return [(int(f[i]), int(c[i]), int(b[i])) for i in range(n.value)]
