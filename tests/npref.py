"""Independent NumPy helpers used by the pins (no code shared with the oracle)."""
import numpy as np


def quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def quat_rot(q):
    """Rotation matrix via q v q* applied to the basis vectors."""
    qc = np.array([q[0], -q[1], -q[2], -q[3]])
    cols = []
    for e in np.eye(3):
        v = quat_mul(quat_mul(q, np.r_[0.0, e]), qc)
        cols.append(v[1:])
    return np.array(cols).T


def signed_svd(F):
    U, s, Vt = np.linalg.svd(F)
    if np.linalg.det(U) < 0:
        U[:, 2] *= -1
        s = s.copy()
        s[2] *= -1
    if np.linalg.det(Vt) < 0:
        Vt[2, :] *= -1
        s = s.copy()
        s[2] *= -1
    return U, s, Vt.T


def lcp_bruteforce(A, q):
    """Solve 0 <= lam  perp  A lam + q >= 0 by enumerating active sets."""
    n = len(q)
    best = None
    for mask in range(1 << n):
        act = [i for i in range(n) if mask >> i & 1]
        lam = np.zeros(n)
        if act:
            Aa = A[np.ix_(act, act)]
            try:
                lam[act] = np.linalg.solve(Aa, -q[act])
            except np.linalg.LinAlgError:
                continue
        w = A @ lam + q
        if (lam >= -1e-12).all() and (w >= -1e-12).all() and abs(lam @ w) < 1e-10:
            if best is not None and not np.allclose(best, lam, atol=1e-9):
                raise AssertionError("LCP solution not unique")
            best = lam
    return best
