"""The single-precision build of the oracle source (oracle/nsn_oracle_f32.c), the
probe the per-row parity tests use to measure what FP32 rounding alone does to each
quantity: it runs the same algorithm (its record agrees with the FP64 build's to
single-precision level on a well-conditioned case) and does round (the records are
not identical)."""
import numpy as np

import scene_inputs as si
from oracle import oracle as O

H = 1.0 / 60.0


def test_f32_probe_runs_the_same_iteration():
    d = si.batched_env(seed=1003, tets_max=150)
    p = O.make_params()
    recs = []
    for k in (1, 2):
        env = O.OracleEnv(d)
        env.set_record(k)
        env.step(H, 3, 30, 0.0, p)
        recs.append(env.record())
    it = {k: recs[1][k] for k in ["lam", "u", "rx", "rq", "px"]}
    prev = {k: recs[0][k] for k in ["lam", "u", "rx", "rq", "px"]}
    e64 = O.OracleEnv(d)
    nc = len(e64.contact_features(H, p)[1])
    st = e64.get_state()
    a = e64.eval_iterate(H, 30, nc, it, prev, p)
    e32 = O.OracleEnvF32(d)
    e32.set_state(st)
    e32.set_time(0.0)
    b = e32.eval_iterate(H, 30, nc, it, prev, p)
    for f in ["err", "cdiag", "P", "b", "Az", "g", "hdiag", "alpha", "active"]:
        x, y = np.asarray(a[f]), np.asarray(b[f])
        assert x.shape == y.shape, f
        rel = np.abs(x - y).max() / (np.abs(x).max() + 1e-30)
        assert rel < 1e-2, (f, rel)
    assert not np.array_equal(a["P"], b["P"])
    assert np.array_equal(a["active"], b["active"])
