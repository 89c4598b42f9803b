"""ctypes front end of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import
this module.  It never imports the GPU package and the GPU package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None
_LIBS = {}

# per-iteration record fields (nsn_oracle.h ORC_REC_*)
REC_FIELDS = ["lam", "u", "rx", "rq", "px", "err", "cdiag", "P", "b", "Az", "dlam", "g", "hdiag",
              "alpha", "rn", "rf", "cblk", "f", "fhat", "uprev", "active", "resid"]

D = C.POINTER(C.c_double)
I32 = C.POINTER(C.c_int32)
I64 = C.POINTER(C.c_int64)


class _Desc(C.Structure):
    _fields_ = [
        ("n_rigid", C.c_int32),
        ("rigid_mass", D), ("rigid_inertia", D), ("rigid_x", D), ("rigid_q", D),
        ("rigid_v", D), ("rigid_w", D), ("rigid_shape", I32), ("rigid_extent", D),
        ("n_particles", C.c_int32),
        ("particle_x", D), ("particle_v", D), ("particle_rest", D), ("particle_mass", D),
        ("n_tets", C.c_int32), ("tet_ids", I32), ("tet_material", D),
        ("n_joints", C.c_int32), ("joint_type", I32), ("joint_body", I32),
        ("joint_anchor", D), ("joint_axis", D), ("joint_ref", D), ("joint_drive", D),
        ("mu", C.c_double), ("gravity", C.c_double * 3), ("ground", C.c_int32),
        ("max_contacts", C.c_int32), ("tet_model", C.c_int32),
    ]


class Params(C.Structure):
    _fields_ = [("ncp", C.c_int32), ("rmode", C.c_int32), ("damping", C.c_double),
                ("eps", C.c_double), ("geo_stiff", C.c_int32), ("fem_mode", C.c_int32),
                ("margin", C.c_double), ("warm", C.c_int32), ("line_search", C.c_int32),
                ("linear", C.c_int32), ("islands", C.c_int32), ("watchdog", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("cr_iters", C.c_int32),
                ("n_contacts", C.c_int32), ("overflow", C.c_int32),
                ("nonfinite", C.c_int32), ("fallback", C.c_int32),
                ("watchdog", C.c_int32), ("pad", C.c_int32),
                ("r_ncp", C.c_double), ("r_contact", C.c_double), ("merit", C.c_double),
                ("r_ncp_first", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


def lib(path=None):
    """The oracle library (built on first use), or the one at `path` (a variant built
    by a test, e.g. with a planted mistake)."""
    global _LIB
    if path is not None:
        if path not in _LIBS:
            _LIBS[path] = _bind(C.CDLL(path))
        return _LIBS[path]
    if _LIB is None:
        path = _build.LIB
        src = _build.SRC
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src) or \
                os.path.getmtime(path) < os.path.getmtime(_build.HDR):
            _build.build()
        _LIB = _bind(C.CDLL(path))
    return _LIB


def _bind(L):
    if True:
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(_Desc), C.c_char_p, C.c_int]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.POINTER(Params), C.c_double, C.c_int, C.c_int,
                               C.c_double, C.POINTER(Stats)]
        L.orc_get_state.argtypes = [C.c_void_p] + [D] * 6
        L.orc_set_state.argtypes = [C.c_void_p] + [D] * 6
        L.orc_get_time.restype = C.c_double
        L.orc_get_time.argtypes = [C.c_void_p]
        L.orc_set_time.argtypes = [C.c_void_p, C.c_double]
        L.orc_num_contacts.argtypes = [C.c_void_p]
        L.orc_num_rows.argtypes = [C.c_void_p]
        L.orc_get_contacts.argtypes = [C.c_void_p, I64, I32, D, D, C.c_int]
        L.orc_get_lambda.argtypes = [C.c_void_p, D]
        L.orc_set_mlp.argtypes = [C.c_void_p, D, C.c_int64]
        L.orc_get_history.argtypes = [C.c_void_p, D, C.c_int]
        L.orc_get_merit_history.argtypes = [C.c_void_p, D, C.c_int]
        L.orc_set_prev.argtypes = [C.c_void_p, C.c_int, I64, D, D]
        L.orc_get_rows_debug.argtypes = [C.c_void_p, D, D, D, C.c_int]
        L.orc_ncp_fb.argtypes = [C.c_double] * 3 + [D] * 3
        L.orc_ncp_min.argtypes = [C.c_double] * 3 + [D] * 3
        L.orc_friction_w.restype = C.c_double
        L.orc_friction_w.argtypes = [C.c_int] + [C.c_double] * 5
        L.orc_svd3.argtypes = [D] * 4
        L.orc_sym_eig3.argtypes = [D] * 3
        L.orc_lame.argtypes = [C.c_double, C.c_double, D, D, D]
        L.orc_neohookean.argtypes = [D, C.c_double, C.c_double, C.c_double, D, D, D]
        L.orc_compliance3.argtypes = [D, C.c_double, C.c_int, D]
        L.orc_linear_tet.argtypes = [D, D, C.c_double, C.c_double, C.c_double, D, D, D, D]
        L.orc_pcr_dense.argtypes = [C.c_int, D, D, D, C.c_int, D, D]
        L.orc_pcg_dense.argtypes = [C.c_int, D, D, D, C.c_int, D, D]
        L.orc_quat_kinematic.argtypes = [D, D]
        L.orc_tangent_basis.argtypes = [D, D, D]
        L.orc_mlp_num_params.restype = C.c_int64
        L.orc_mlp_forward.argtypes = [D, C.c_int64, D, D]
        L.orc_mlp_loss_grad.restype = C.c_double
        L.orc_mlp_loss_grad.argtypes = [D, C.c_int64, D, D, D]
        L.orc_mlp_loss_grad_bf16.restype = C.c_double
        L.orc_mlp_loss_grad_bf16.argtypes = [D, C.c_int64, D, D, D]
        L.orc_mlp_preact_bf16.argtypes = [D, D, D]
        L.orc_contact_features.argtypes = [C.c_void_p, C.POINTER(Params), C.c_double, D, I64, C.c_int]
        L.orc_set_record.argtypes = [C.c_void_p, C.c_int]
        L.orc_get_record.argtypes = [C.c_void_p, C.c_int, D, C.c_int]
        L.orc_eval_iterate.argtypes = [C.c_void_p, C.POINTER(Params), C.c_double, C.c_int, C.c_int] + [D] * 10
    return L


def _d(a):
    return a.ctypes.data_as(D)


def _i32(a):
    return a.ctypes.data_as(I32)


def make_params(sp=None, **kw):
    """Oracle parameter struct from a scene_inputs.SolverParams (or keywords)."""
    vals = dict(ncp=0, rmode=2, damping=0.75, eps=1e-6, geo_stiff=1, fem_mode=0,
                margin=5e-3, warm=0, line_search=0, linear=0, islands=0, watchdog=0)
    if sp is not None:
        for k in vals:
            vals[k] = getattr(sp, k)
    vals.update(kw)
    return Params(**vals)


class OracleEnv:
    """One environment stepped by the FP64 oracle (lib_path: a variant of the library,
    for tests that plant a mistake in it)."""

    def __init__(self, desc, lib_path=None):
        self.desc = desc
        self._lib = lib(lib_path)
        L = self._lib
        self._keep = {}

        def arr(name, dtype):
            a = np.ascontiguousarray(getattr(desc, name), dtype=dtype).ravel()
            if a.size == 0:
                a = np.zeros(1, dtype=dtype)
            self._keep[name] = a
            return a

        s = _Desc()
        s.n_rigid = desc.n_rigid
        for name in ["rigid_mass", "rigid_inertia", "rigid_x", "rigid_q", "rigid_v", "rigid_w",
                     "rigid_extent", "particle_x", "particle_v", "particle_rest", "particle_mass",
                     "tet_material", "joint_anchor", "joint_axis", "joint_ref", "joint_drive"]:
            setattr(s, name, _d(arr(name, np.float64)))
        for name in ["rigid_shape", "tet_ids", "joint_type", "joint_body"]:
            setattr(s, name, _i32(arr(name, np.int32)))
        s.n_particles = desc.n_particles
        s.n_tets = desc.n_tets
        s.n_joints = desc.n_joints
        s.mu = desc.mu
        s.gravity = (C.c_double * 3)(*desc.gravity)
        s.ground = desc.ground
        s.max_contacts = desc.max_contacts
        s.tet_model = int(getattr(desc, "tet_model", 0))
        err = C.create_string_buffer(256)
        self.h = L.orc_create(C.byref(s), err, 256)
        if not self.h:
            raise ValueError(err.value.decode())
        self.nr, self.np_ = desc.n_rigid, desc.n_particles

    def __del__(self):
        if getattr(self, "h", None):
            self._lib.orc_destroy(self.h)
            self.h = None

    def step(self, h, newton_iters, cr_iters, tol=0.0, params=None):
        p = params if params is not None else make_params()
        st = Stats()
        self._lib.orc_step(self.h, C.byref(p), float(h), int(newton_iters), int(cr_iters), float(tol),
                       C.byref(st))
        return st.as_dict()

    def get_state(self):
        rx = np.zeros((self.nr, 3)); rq = np.zeros((self.nr, 4)); rv = np.zeros((self.nr, 3))
        rw = np.zeros((self.nr, 3)); px = np.zeros((self.np_, 3)); pv = np.zeros((self.np_, 3))
        self._lib.orc_get_state(self.h, _d(rx), _d(rq), _d(rv), _d(rw), _d(px), _d(pv))
        return dict(rigid_x=rx, rigid_q=rq, rigid_v=rv, rigid_w=rw, particle_x=px, particle_v=pv)

    def set_state(self, st):
        g = lambda k, shape: np.ascontiguousarray(st[k], dtype=np.float64).reshape(shape)
        rx, rq, rv, rw = (g("rigid_x", (self.nr, 3)), g("rigid_q", (self.nr, 4)),
                          g("rigid_v", (self.nr, 3)), g("rigid_w", (self.nr, 3)))
        px, pv = g("particle_x", (self.np_, 3)), g("particle_v", (self.np_, 3))
        self._lib.orc_set_state(self.h, _d(rx), _d(rq), _d(rv), _d(rw), _d(px), _d(pv))

    @property
    def time(self):
        return self._lib.orc_get_time(self.h)

    @time.setter
    def time(self, t):
        self._lib.orc_set_time(self.h, float(t))

    def contacts(self):
        n = self._lib.orc_num_contacts(self.h)
        key = np.zeros(max(n, 1), np.int64); bodies = np.zeros((max(n, 1), 2), np.int32)
        geom = np.zeros((max(n, 1), 10)); lam = np.zeros((max(n, 1), 3))
        self._lib.orc_get_contacts(self.h, key.ctypes.data_as(I64), _i32(bodies), _d(geom), _d(lam), n)
        return dict(key=key[:n], bodies=bodies[:n], normal=geom[:n, 0:3], a_local=geom[:n, 3:6],
                    b_local=geom[:n, 6:9], thickness=geom[:n, 9], lam=lam[:n])

    def lambdas(self):
        n = self._lib.orc_num_rows(self.h)
        out = np.zeros(max(n, 1))
        self._lib.orc_get_lambda(self.h, _d(out))
        return out[:n]

    def history(self):
        out = np.zeros(256)
        n = self._lib.orc_get_history(self.h, _d(out), 256)
        return out[:n]

    def set_prev(self, keys, lam3, lam_joint):
        """Previous-step contact multipliers by key (ascending) and joint multipliers."""
        k = np.ascontiguousarray(keys, dtype=np.int64)
        l3 = np.ascontiguousarray(lam3, dtype=np.float64).reshape(-1)
        lj = np.ascontiguousarray(lam_joint, dtype=np.float64).reshape(-1)
        self._keep["prev"] = (k, l3, lj)
        assert lj.size == 6 * self.desc.n_joints
        st = self._lib.orc_set_prev(self.h, k.size, k.ctypes.data_as(I64), _d(l3), _d(lj) if lj.size else None)
        if st != 0:
            raise ValueError("orc_set_prev: bad keys or count")

    def merit_history(self):
        out = np.zeros(256)
        n = self._lib.orc_get_merit_history(self.h, _d(out), 256)
        return out[:n]

    def rows_debug(self):
        n = self._lib.orc_num_rows(self.h)
        e, c, p = np.zeros(max(n, 1)), np.zeros(max(n, 1)), np.zeros(max(n, 1))
        self._lib.orc_get_rows_debug(self.h, _d(e), _d(c), _d(p), n)
        return e[:n], c[:n], p[:n]

    def set_mlp(self, blob):
        if blob is None:
            self._lib.orc_set_mlp(self.h, None, 0)
            return
        b = np.ascontiguousarray(blob, dtype=np.float64)
        self._keep["mlp"] = b
        self._lib.orc_set_mlp(self.h, _d(b), b.size)

    def set_record(self, k):
        """Record Newton iteration k of the following steps (-1: off)."""
        self._lib.orc_set_record(self.h, int(k))

    def record(self):
        """The recorded iteration: {field: array} (oracle row order: joints, contacts,
        tets); empty arrays for fields the iteration did not reach."""
        out = {}
        for i, name in enumerate(REC_FIELDS):
            n = self._lib.orc_get_record(self.h, i, None, 0)
            a = np.zeros(max(n, 1))
            if n > 0:
                self._lib.orc_get_record(self.h, i, _d(a), n)
            out[name] = a[:max(n, 0)]
        return out

    def eval_iterate(self, h, M, n_contacts, it, prev=None, params=None):
        """One Newton iteration at a given iterate from the env's current state (q^-,
        u^-): it = dict(lam, u, rx, rq, px) (oracle row order, u = 6 per rigid body then
        3 per particle); prev: the previous iterate (same keys) for the secant, or None.
        Returns record() of that iteration."""
        p = params if params is not None else make_params()
        f = lambda a: np.ascontiguousarray(a, np.float64).ravel()
        cur = [f(it[k]) for k in ["lam", "u", "rx", "rq", "px"]]
        cur = [a if a.size else np.zeros(1) for a in cur]
        self._keep["inj"] = cur
        if prev is not None:
            pv = [f(prev[k]) for k in ["lam", "u", "rx", "rq", "px"]]
            pv = [a if a.size else np.zeros(1) for a in pv]
            self._keep["inj_p"] = pv
            pptr = [_d(a) for a in pv]
        else:
            pptr = [None] * 5
        rc = self._lib.orc_eval_iterate(self.h, C.byref(p), float(h), int(M), int(n_contacts),
                                        *[_d(a) for a in cur], *pptr)
        if rc == -2:
            raise ValueError("orc_eval_iterate: the contact set at q^- differs from the caller's")
        if rc not in (0, -4):
            raise ValueError(f"orc_eval_iterate failed ({rc})")
        return self.record()

    def contact_features(self, h, params=None):
        p = params if params is not None else make_params()
        cap = self.desc.max_contacts
        feat = np.zeros((max(cap, 1), 12)); key = np.zeros(max(cap, 1), np.int64)
        n = self._lib.orc_contact_features(self.h, C.byref(p), float(h), _d(feat), key.ctypes.data_as(I64), cap)
        n = min(n, cap)
        return feat[:n], key[:n]


# ---------------------------------------------------------------------------
# primitives (for pins)
# ---------------------------------------------------------------------------

def ncp_fb(Cn, lam, r):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    lib().orc_ncp_fb(Cn, lam, r, C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def ncp_min(Cn, lam, r):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    lib().orc_ncp_min(Cn, lam, r, C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def friction_w(ncp, vnorm, lam_n, lamf_norm, mu, r):
    return lib().orc_friction_w(int(ncp), vnorm, lam_n, lamf_norm, mu, r)


def svd3(F):
    F = np.ascontiguousarray(F, np.float64).reshape(9)
    U, s, V = np.zeros(9), np.zeros(3), np.zeros(9)
    lib().orc_svd3(_d(F), _d(U), _d(s), _d(V))
    return U.reshape(3, 3), s, V.reshape(3, 3)


def sym_eig3(A):
    A = np.ascontiguousarray(A, np.float64).reshape(9)
    Q, w = np.zeros(9), np.zeros(3)
    lib().orc_sym_eig3(_d(A), _d(Q), _d(w))
    return Q.reshape(3, 3), w


def lame(E, nu):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    lib().orc_lame(E, nu, C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def neohookean(s, C1, D1, alpha):
    s = np.ascontiguousarray(s, np.float64)
    psi, g, H = C.c_double(), np.zeros(3), np.zeros(9)
    lib().orc_neohookean(_d(s), C1, D1, alpha, C.byref(psi), _d(g), _d(H))
    return psi.value, g, H.reshape(3, 3)


def compliance3(H, floor_, mode=0):
    H = np.ascontiguousarray(H, np.float64).reshape(9)
    E = np.zeros(9)
    lib().orc_compliance3(_d(H), floor_, int(mode), _d(E))
    return E.reshape(3, 3)


def linear_tet(Dminv, x, E, nu, Ve):
    """Linear tet of Sec. 9.2 at node positions x (4 x 3): strains (xx yy zz yz xz xy),
    rows ds/dx (6 x 4 x 3), stress V_e K_e s and compliance (V_e K_e)^-1 (6 x 6)."""
    Dm = np.ascontiguousarray(Dminv, np.float64).reshape(9)
    x = np.ascontiguousarray(x, np.float64).reshape(12)
    eps, rows, c, Cm = np.zeros(6), np.zeros(72), np.zeros(6), np.zeros(36)
    lib().orc_linear_tet(_d(Dm), _d(x), E, nu, Ve, _d(eps), _d(rows), _d(c), _d(Cm))
    return eps, rows.reshape(6, 4, 3), c, Cm.reshape(6, 6)


def pcg_dense(A, b, P, iters):
    A = np.ascontiguousarray(A, np.float64)
    n = A.shape[0]
    b = np.ascontiguousarray(b, np.float64)
    P = np.ascontiguousarray(P, np.float64)
    x, hist = np.zeros(n), np.zeros(max(iters, 1))
    done = lib().orc_pcg_dense(n, _d(A), _d(b), _d(P), int(iters), _d(x), _d(hist))
    return x, hist[:done]


def pcr_dense(A, b, P, iters):
    A = np.ascontiguousarray(A, np.float64)
    n = A.shape[0]
    b = np.ascontiguousarray(b, np.float64)
    P = np.ascontiguousarray(P, np.float64)
    x, hist = np.zeros(n), np.zeros(max(iters, 1))
    done = lib().orc_pcr_dense(n, _d(A), _d(b), _d(P), int(iters), _d(x), _d(hist))
    return x, hist[:done]


def quat_kinematic(q):
    q = np.ascontiguousarray(q, np.float64)
    Q = np.zeros(12)
    lib().orc_quat_kinematic(_d(q), _d(Q))
    return Q.reshape(4, 3)


def tangent_basis(n):
    n = np.ascontiguousarray(n, np.float64)
    d1, d2 = np.zeros(3), np.zeros(3)
    lib().orc_tangent_basis(_d(n), _d(d1), _d(d2))
    return d1, d2


def mlp_num_params():
    return int(lib().orc_mlp_num_params())


def mlp_forward(w, x):
    w = np.ascontiguousarray(w, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 12)
    y = np.zeros((x.shape[0], 3))
    lib().orc_mlp_forward(_d(w), x.shape[0], _d(x), _d(y))
    return y


def mlp_loss_grad(w, x, t):
    w = np.ascontiguousarray(w, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 12)
    t = np.ascontiguousarray(t, np.float64).reshape(-1, 3)
    g = np.zeros_like(w)
    loss = lib().orc_mlp_loss_grad(_d(w), x.shape[0], _d(x), _d(t), _d(g))
    return loss, g


def mlp_loss_grad_bf16(w, x, t):
    """Loss and gradient with every product operand rounded to bfloat16."""
    w = np.ascontiguousarray(w, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 12)
    t = np.ascontiguousarray(t, np.float64).reshape(-1, 3)
    g = np.zeros_like(w)
    loss = lib().orc_mlp_loss_grad_bf16(_d(w), x.shape[0], _d(x), _d(t), _d(g))
    return loss, g


def mlp_preact_bf16(w, x):
    """Pre-activations [n, 3, 64] of the bfloat16-rounded forward pass."""
    w = np.ascontiguousarray(w, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 12)
    out = np.zeros((x.shape[0], 3, 64))
    for s in range(x.shape[0]):
        row = np.ascontiguousarray(x[s])
        lib().orc_mlp_preact_bf16(_d(w), _d(row), _d(out[s]))
    return out


# ---------------------------------------------------------------------------
# The single-precision build of the same source (nsn_oracle_f32.c): a probe of what
# FP32 rounding alone does to each quantity of an iteration.  Only the calls the
# per-row parity tests need are bound.
# ---------------------------------------------------------------------------
F = C.POINTER(C.c_float)


class _DescF32(C.Structure):
    _fields_ = [(n, F if t is D else (C.c_float if t is C.c_double else
                                     (C.c_float * 3 if n == "gravity" else t)))
                for n, t in _Desc._fields_]


class _ParamsF32(C.Structure):
    _fields_ = [(n, C.c_float if t is C.c_double else t) for n, t in Params._fields_]


_LIB_F32 = None


def lib_f32():
    global _LIB_F32
    if _LIB_F32 is None:
        path = _build.LIB_F32
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC) or \
                os.path.getmtime(path) < os.path.getmtime(_build.HDR):
            _build.build_f32()
        L = C.CDLL(path)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(_DescF32), C.c_char_p, C.c_int]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_state.argtypes = [C.c_void_p] + [F] * 6
        L.orc_set_time.argtypes = [C.c_void_p, C.c_float]
        L.orc_get_record.argtypes = [C.c_void_p, C.c_int, F, C.c_int]
        L.orc_eval_iterate.argtypes = [C.c_void_p, C.POINTER(_ParamsF32), C.c_float, C.c_int, C.c_int] + [F] * 10
        _LIB_F32 = L
    return _LIB_F32


class OracleEnvF32:
    """One environment in the single-precision build: state, time and the evaluation
    of one Newton iteration at a given iterate (see OracleEnv.eval_iterate)."""

    def __init__(self, desc):
        self.desc = desc
        self._lib = L = lib_f32()
        self._keep = {}
        s = _DescF32()
        for name, t in _DescF32._fields_:
            if t is F:
                a = np.ascontiguousarray(getattr(desc, name), np.float32).ravel()
                a = a if a.size else np.zeros(1, np.float32)
                self._keep[name] = a
                setattr(s, name, a.ctypes.data_as(F))
            elif t is I32:
                a = np.ascontiguousarray(getattr(desc, name), np.int32).ravel()
                a = a if a.size else np.zeros(1, np.int32)
                self._keep[name] = a
                setattr(s, name, a.ctypes.data_as(I32))
        s.n_rigid, s.n_particles, s.n_tets, s.n_joints = desc.n_rigid, desc.n_particles, desc.n_tets, desc.n_joints
        s.mu = desc.mu
        s.gravity = (C.c_float * 3)(*desc.gravity)
        s.ground, s.max_contacts = desc.ground, desc.max_contacts
        s.tet_model = int(getattr(desc, "tet_model", 0))
        err = C.create_string_buffer(256)
        self.h = L.orc_create(C.byref(s), err, 256)
        if not self.h:
            raise ValueError(err.value.decode())

    def __del__(self):
        if getattr(self, "h", None):
            self._lib.orc_destroy(self.h)
            self.h = None

    def set_state(self, st):
        d = self.desc
        shapes = [("rigid_x", 3 * d.n_rigid), ("rigid_q", 4 * d.n_rigid), ("rigid_v", 3 * d.n_rigid),
                  ("rigid_w", 3 * d.n_rigid), ("particle_x", 3 * d.n_particles), ("particle_v", 3 * d.n_particles)]
        arrs = []
        for k, n in shapes:
            a = np.ascontiguousarray(st[k], np.float32).ravel() if n else np.zeros(1, np.float32)
            arrs.append(a)
        self._keep["state"] = arrs
        self._lib.orc_set_state(self.h, *[a.ctypes.data_as(F) for a in arrs])

    def set_time(self, t):
        self._lib.orc_set_time(self.h, float(t))

    def eval_iterate(self, h, M, n_contacts, it, prev=None, params=None):
        p = params if params is not None else make_params()
        pf = _ParamsF32(**{n: getattr(p, n) for n, _ in Params._fields_})
        f = lambda a: np.ascontiguousarray(a, np.float32).ravel()
        cur = [f(it[k]) for k in ["lam", "u", "rx", "rq", "px"]]
        cur = [a if a.size else np.zeros(1, np.float32) for a in cur]
        self._keep["inj"] = cur
        pptr = [None] * 5
        if prev is not None:
            pv = [f(prev[k]) for k in ["lam", "u", "rx", "rq", "px"]]
            pv = [a if a.size else np.zeros(1, np.float32) for a in pv]
            self._keep["inj_p"] = pv
            pptr = [a.ctypes.data_as(F) for a in pv]
        rc = self._lib.orc_eval_iterate(self.h, C.byref(pf), float(h), int(M), int(n_contacts),
                                        *[a.ctypes.data_as(F) for a in cur], *pptr)
        if rc == -2:
            raise ValueError("orc_eval_iterate (f32): the contact set at q^- differs from the caller's")
        if rc not in (0, -4):
            raise ValueError(f"orc_eval_iterate (f32) failed ({rc})")
        out = {}
        for i, name in enumerate(REC_FIELDS):
            n = self._lib.orc_get_record(self.h, i, None, 0)
            a = np.zeros(max(n, 1), np.float32)
            if n > 0:
                self._lib.orc_get_record(self.h, i, a.ctypes.data_as(F), n)
            out[name] = a[:max(n, 0)].astype(np.float64)
        return out
