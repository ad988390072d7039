"""The DIRK(3,3) x Newton stage driver over the C ABI against the oracle's
time step on a small periodic Taylor-Green case."""
import numpy as np
import pytest

from gpu_common import make_pair, to_dev, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", [dict(dim=2, n_elem=4, m=2, p=2, periodic=True, mach=0.1, Re=100.0),
                                  dict(dim=2, n_elem=4, m=2, p=1, periodic=False, state="shear", mach=0.2),
                                  dict(dim=2, n_elem=4, m=2, p=2, periodic=True, mach=0.1, Re=100.0, supg=True)])
def test_dirk_step_matches_oracle(case):
    from oracle.newton import dirk_step
    from paper_2402_11361_amd.driver import StageDriver, alexander_dirk33
    from oracle import dirk
    say(f"[driver] {case}")
    case = dict(case)
    supg = case.pop("supg", False)
    S, inp, ctx = make_pair(case, supg=supg)
    A, b, c = alexander_dirk33()
    Ao, bo, co = dirk.dirk33()
    assert np.allclose(A, Ao, rtol=0, atol=1e-14)
    drv = StageDriver(ctx, rtol=1e-13, newton_abs=1e-12, newton_rel=1e-12, max_newton=12)
    q, u, uh = to_dev(inp["q"]), to_dev(inp["u"]), to_dev(inp["uh"])
    infos = drv.step(q, u, uh, inp["dt"])
    qo, uo, uho, oinfos = dirk_step(S, inp["q"], inp["u"], inp["uh"], inp["dt"],
                                   newton_kw=dict(abs_tol=1e-12, rel_tol=1e-12, max_it=12))
    for st in infos:
        assert st["res_hist"][-1] < 1e-11, st["res_hist"]
    du = np.abs(u.cpu().numpy() - uo).max() / np.abs(uo).max()
    duh = np.abs(uh.cpu().numpy() - uho).max() / np.abs(uho).max()
    dq = np.abs(q.cpu().numpy() - qo).max() / max(np.abs(qo).max(), 1e-30)
    assert du < 1e-10 and duh < 1e-10 and dq < 1e-8, (du, duh, dq)
    # the step changed the state (not a trivial pass)
    assert np.abs(uo - inp["u"]).max() > 1e-6
