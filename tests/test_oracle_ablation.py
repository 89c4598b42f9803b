"""The heavy-stack ablation (complementarity preconditioning and linear solver) on the
FP64 oracle: the qualitative claims of the paper's rigid tests and solver study.

Stack of five cubes of 8, 64, ..., 32768 kg (4096:1), mu = 0.5, h = 1/60, Fischer-
Burmeister, 10 Newton x 40 linear iterations per step, 30 steps from rest.
  * r = h^2 * effective mass with PCR holds the stack (contact residual <= 1e-2);
  * identity scaling and the constant h^2 let it collapse;
  * with the same truncated budget PCG ends far above PCR (non-monotone residual)."""
import numpy as np

import scene_inputs as si
from oracle import oracle as O
from scene_inputs.scenes import heavy_stack


def run(rmode, linear, steps=30):
    d = heavy_stack(seed=0)
    e = O.OracleEnv(d)
    rc = []
    for _ in range(steps):
        st = e.step(1 / 60, 10, 40, 0.0, O.make_params(rmode=rmode, ncp=si.NCP_FB, linear=linear))
        rc.append(st["r_contact"])
    S = e.get_state()
    rest = 0.05 + 0.1 * np.arange(d.n_rigid)
    sink = float(max(0.0, (rest - S["rigid_x"][:, 2]).max()))
    return float(np.median(rc)), sink


def test_heavy_stack_needs_effective_mass_scaling_and_pcr():
    good_r, good_sink = run(si.RMODE_H2_EFFMASS, 0)
    assert good_r <= 1e-2 and good_sink < 1e-3, (good_r, good_sink)
    for rmode in [si.RMODE_IDENTITY, si.RMODE_H2]:
        r, sink = run(rmode, 0)
        assert r > 100 * good_r and sink > 0.05, (rmode, r, sink)
    pcg_r, _ = run(si.RMODE_H2_EFFMASS, 1)
    assert pcg_r > 100 * good_r, (pcg_r, good_r)


def test_geometric_stiffness_keeps_stretched_sheet_converging():
    """Sec. 8.3 / the stretched-sheet merit figure: as the sheet is pulled to large
    strain, the diagonal geometric stiffness keeps the damped Newton iteration close to
    the solution; without it the iterates overshoot (larger residuals from the first
    steps on, growing by orders of magnitude)."""
    d = si.stretched_sheet()
    res = {}
    for gs in [1, 0]:
        e = O.OracleEnv(d)
        r = []
        for _ in range(8):
            st = e.step(1 / 60, 30, 60, 1e-6, O.make_params(geo_stiff=gs))
            r.append(st["r_ncp"])
        res[gs] = float(np.median(r))
    assert res[1] < 1e-2 and res[0] > 1.0, res
