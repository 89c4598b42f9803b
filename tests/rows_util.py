"""Per-row comparison of one Newton iteration between the HIP path and the FP64 oracle,
from identical iterates.

The GPU runs a dump step (nsn_dump_iteration) on a contact set injected from the
oracle (nsn_set_contacts); its iterate k (and k-1, for the secant of the geometric
stiffness) is handed to the oracle's evaluation at a given iterate
(orc_eval_iterate), and every per-row and per-DOF quantity of that iteration is
compared element by element.

Tolerance of an element: the larger of
  * 1e-4 of the largest oracle value of its group (rows or DOFs of one kind and unit:
    the joint rows by joint type and row index, tet rows, contact normal rows,
    friction rows; rigid linear, rigid angular and particle DOFs);
  * 10x the element's FP32 conditioning, measured on the oracle itself as the larger
    of (a) how far the FP64 value moves when the iterate and the pre-step state are
    perturbed at the level of FP32 rounding (three trials) and (b) how far the same
    source evaluated in single precision (oracle/nsn_oracle_f32.c) lies from the FP64
    value on the same inputs, at the given iterate and at each perturbed one -- the
    rounding of the arithmetic itself, which input perturbations miss where terms
    cancel (a body at rest: g is a sum of large opposite momenta; a friction row near
    its inactive limit: den of W cancels).  Its error at a cancellation is one draw
    from a wide distribution, so it is sampled at several nearby inputs.
Elements whose tolerance exceeds 1e-3 of their group's scale are counted as
ill-conditioned in the report (a kink of the NCP function inside the rounding band,
a friction row switching activity, a repeated singular value); they are compared at
their own tolerance like every other element.
"""
import numpy as np

from oracle import oracle as O

FP32_REL = 1.2e-7
BASE_TOL = 1e-4
CAP = 1e-3
SPREAD_FACTOR = 10.0

# fields compared (the oracle record name -> the GPU dump name)
ROW_FIELDS = [("err", "err"), ("cdiag", "cdiag"), ("P", "P"), ("b", "b"), ("Az", "Az")]


def row_maps(desc, nc):
    """(gpu_to_orc row index array, group label per oracle row) for an env with nc
    contacts.  GPU rows: joints | tets | contacts; oracle rows: joints | contacts | tets."""
    nj, nt = desc.n_joints, desc.n_tets
    tr = 6 if getattr(desc, "tet_model", 0) == 1 else 3
    gj = np.arange(6 * nj)
    gt = 6 * nj + np.arange(tr * nt)
    gc = 6 * nj + tr * nt + np.arange(3 * nc)
    g2o = np.empty(6 * nj + tr * nt + 3 * nc, np.int64)
    g2o[gj] = gj
    g2o[gc] = 6 * nj + np.arange(3 * nc)
    g2o[gt] = 6 * nj + 3 * nc + np.arange(tr * nt)
    group = np.empty(g2o.size, object)
    jt = np.asarray(desc.joint_type).ravel()
    # units differ by row: positional rows (m/s), orientation rows (rad/s), the drive row
    kinds = {0: ["lin"] * 3 + ["ang"] * 2 + ["drive"], 1: ["lin"] * 2 + ["ang"] * 3 + ["drive"]}
    for j in range(nj):
        for r in range(6):
            group[6 * j + r] = f"{'prismatic' if int(jt[j]) == 1 else 'revolute'}_{kinds[int(jt[j])][r]}"
    for i in range(nc):
        group[6 * nj + 3 * i] = "normal"
        group[6 * nj + 3 * i + 1:6 * nj + 3 * i + 3] = "friction"
    group[6 * nj + 3 * nc:] = "tet"
    return g2o, group


def dof_groups(desc):
    g = np.empty(6 * desc.n_rigid + 3 * desc.n_particles, object)
    for i in range(desc.n_rigid):
        g[6 * i:6 * i + 3] = "rigid_lin"
        g[6 * i + 3:6 * i + 6] = "rigid_ang"
    g[6 * desc.n_rigid:] = "particle"
    return g


def oracle_contacts(desc, pre, h, params):
    """The oracle's contact list at the pre-step state (collision detection only)."""
    oe = O.OracleEnv(desc)
    oe.set_state({k: np.asarray(v, np.float64) for k, v in pre.items() if k != "time"})
    oe.time = pre["time"]
    oe.step(h, 0, 0, 0.0, params)
    return oe.contacts()


def inject(scene, env, con):
    scene.set_contacts(env, con["key"], con["bodies"], con["normal"], con["a_local"], con["b_local"],
                       con["thickness"])


def gpu_iterate(dump, desc, nc, prev=False):
    """The GPU's iterate in the oracle's layouts (rows reordered)."""
    g2o, _ = row_maps(desc, nc)
    p = "prev_" if prev else ""
    lam = np.zeros(g2o.size)
    lam[g2o] = dump[p + "lam"]
    return dict(lam=lam, u=np.asarray(dump[p + "u"], np.float64), rx=np.asarray(dump[p + "rx"], np.float64),
                rq=np.asarray(dump[p + "rq"], np.float64), px=np.asarray(dump[p + "px"], np.float64))


def _perturb(it, rng, h):
    out = {}
    for k, v in it.items():
        v = np.asarray(v, np.float64)
        if v.size == 0:
            out[k] = v
            continue
        w = v * (1.0 + FP32_REL * rng.standard_normal(v.shape))
        if k == "u":
            w = w + FP32_REL * 9.81 * h * rng.standard_normal(v.shape)
        if k == "lam":
            w = w + FP32_REL * (np.abs(v).max() + 1e-30) * 1e-3 * rng.standard_normal(v.shape)
        out[k] = w
    return out


def _perturb_state(pre, rng, h):
    st = {}
    for k, v in pre.items():
        if k == "time":
            continue
        v = np.asarray(v, np.float64)
        if v.size == 0:
            st[k] = v
            continue
        w = v * (1.0 + FP32_REL * rng.standard_normal(v.shape))
        if k.endswith(("_v", "_w")):
            w = w + FP32_REL * 9.81 * h * rng.standard_normal(v.shape)
        st[k] = w
    return st


def oracle_eval(desc, pre_state, time, h, M, nc, it, prev, params):
    oe = O.OracleEnv(desc)
    oe.set_state(pre_state)
    oe.time = time
    return oe.eval_iterate(h, M, nc, it, prev, params)


def compare_iteration(scene, env, desc, pre, h, k, M, params, trials=3, seed=0):
    """Compare the last dump step of `env` with the oracle's evaluation at the GPU's
    iterate.  Returns ({field/group: dict(err, n, illcond, tol_max)}, [messages of
    elements above their tolerance]); err and tol_max are relative to the group's
    scale."""
    dump = scene.read_iteration(env)
    nc = len(dump["alpha"])
    it = gpu_iterate(dump, desc, nc)
    prev = gpu_iterate(dump, desc, nc, prev=True) if k >= 1 else None
    pre_state = {kk: np.asarray(v, np.float64) for kk, v in pre.items() if kk != "time"}
    base = oracle_eval(desc, pre_state, pre["time"], h, M, nc, it, prev, params)
    fields = ["err", "cdiag", "P", "b", "Az", "g", "hdiag", "alpha", "active", "cblk", "dlam"]
    rng = np.random.default_rng(seed)
    spreads = {f: np.zeros(np.asarray(base[f]).shape) for f in fields}
    f32_note = ""

    def widen(rec, ref):
        for f in fields:
            spreads[f] = np.maximum(spreads[f], np.abs(np.asarray(rec[f]) - np.asarray(ref[f])))

    def f32_eval(st, itp, prevp):
        # the arithmetic's own rounding: the single-precision build on the same inputs
        nonlocal f32_note
        try:
            o32 = O.OracleEnvF32(desc)
            o32.set_state(st)
            o32.set_time(pre["time"])
            return o32.eval_iterate(h, M, nc, itp, prevp, params)
        except ValueError as ex:  # its collision detection found another contact set
            f32_note = f" (single-precision probe unavailable: {ex})"
            return None

    rec = f32_eval(pre_state, it, prev)
    if rec is not None:
        widen(rec, base)
    for _ in range(trials):
        st = _perturb_state(pre, rng, h)
        itp = _perturb(it, rng, h)
        prevp = _perturb(prev, rng, h) if prev is not None else None
        rec = oracle_eval(desc, st, pre["time"], h, M, nc, itp, prevp, params)
        widen(rec, base)
        # one more sample of the single-precision rounding, at this nearby input: at a
        # cancellation one sample can fall far below another evaluation order's error
        rec32 = f32_eval(st, itp, prevp)
        if rec32 is not None:
            widen(rec32, rec)
    g2o, rgroup = row_maps(desc, nc)
    report = {}
    bad = []

    def check(name, gpu, orc, spread, groups):
        gpu = np.asarray(gpu, np.float64).ravel()
        orc = np.asarray(orc, np.float64).ravel()
        spread = np.asarray(spread, np.float64).ravel()
        groups = np.asarray(groups, object).ravel()
        for grp in sorted(set(groups)):
            m = groups == grp
            if not m.any():
                continue
            scale = np.abs(orc[m]).max()
            if scale == 0.0:
                scale = 1e-30
            err = np.abs(gpu[m] - orc[m])
            tol = np.maximum(BASE_TOL * scale, SPREAD_FACTOR * spread[m])
            report[f"{name}/{grp}"] = dict(err=float((err / scale).max()), n=int(m.sum()),
                                           illcond=int((tol > CAP * scale).sum()),
                                           tol_max=float((tol / scale).max()))
            over = err > tol
            if over.any():
                i = np.flatnonzero(m)[np.flatnonzero(over)[0]]
                bad.append(f"{name}/{grp}: {int(over.sum())} of {int(m.sum())} elements above tolerance; "
                           f"first at {i}: gpu {gpu[i]:.6e} oracle {orc[i]:.6e} (scale {scale:.3e}, "
                           f"spread {spread[i]:.3e}){f32_note}")

    for orc_name, gpu_name in ROW_FIELDS:
        orc = np.asarray(base[orc_name])
        check(orc_name, dump[gpu_name], orc[g2o], spreads[orc_name][g2o], rgroup[g2o])
    check("g", dump["g"], base["g"], spreads["g"], dof_groups(desc))
    if desc.n_particles:
        check("hdiag", dump["hdiag"], base["hdiag"], spreads["hdiag"], np.full(3 * desc.n_particles, "particle", object))
    if nc:
        cg = np.full(nc, "contact", object)
        check("alpha", dump["alpha"], base["alpha"], spreads["alpha"], cg)
        check("active", dump["active"], base["active"], spreads["active"], cg)
    if desc.n_tets and getattr(desc, "tet_model", 0) == 0:
        nj = desc.n_joints
        r0 = 6 * nj + 3 * nc + 3 * np.arange(desc.n_tets)  # oracle first row of every tet
        cb = np.asarray(base["cblk"]).reshape(-1, 9)[r0]
        sb = np.asarray(spreads["cblk"]).reshape(-1, 9)[r0]
        pick = [0, 4, 8, 1, 2, 5]  # xx yy zz xy xz yz of the 3x3 block
        check("tetC", np.asarray(dump["tetc"]).ravel(), cb[:, pick].ravel(), sb[:, pick].ravel(),
              np.full(6 * desc.n_tets, "tet", object))
    # the solve itself (M linear iterations): reported, not asserted -- Krylov iterates
    # amplify rounding through the scalars one PCR shares over the env (Sec. 11)
    dl = np.asarray(base["dlam"])[g2o]
    sc_ = np.abs(dl).max() + 1e-30
    report["dlam(report only)"] = dict(err=float(np.abs(np.asarray(dump["dlam"], np.float64) - dl).max() / sc_),
                                       n=int(dl.size), illcond=0, tol_max=0.0)
    return report, bad
