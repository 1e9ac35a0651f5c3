"""The walk-log reconstruction the GPU parity tests rely on, checked on the
CPU against the oracle alone: S rebuilt from the oracle's own log (status,
terminal triangle, FP32 barycentrics) equals the oracle's estimate to the
rounding of those barycentrics, for the interior, exterior and jump-only
forms; one walk's terminal triangle changed in the log is detected."""
import numpy as np
import pytest

from paper_2606_05581_amd import workloads as W
from parity_util import reconstruct_from_log


@pytest.fixture(scope="module")
def soup_case():
    wl = W.soup8_53k(N=120, walks=32)
    return wl.cases[0], wl.walks


@pytest.mark.parametrize("exterior,jump_only", [(False, False), (True, False), (True, True)])
def test_oracle_estimate_equals_its_log(oracle_mod, soup_case, exterior, jump_only):
    case, walks = soup_case
    sc = oracle_mod.Scene(case.V, case.F, bvh=True)
    r = oracle_mod.estimate(sc, case.rows, case.basis, walks, case.eps, case.h, exterior=exterior, log=True,
                            nthreads=4, jump_only=jump_only)
    S, _ = oracle_mod.finalize(r["acc"], r["acc2"], case.rows.w, case.h, walks, r["discarded"])
    Sr = reconstruct_from_log(oracle_mod, case, r["log_status"], r["log_tri"], r["log_bary"], exterior, jump_only)
    assert np.abs(S - Sr).max() <= 1e-7 * np.abs(S).max()
    if exterior:
        assert r["n_escaped"].sum() > 0  # the escaped-walk branch is exercised


def test_a_changed_walk_is_detected(oracle_mod, soup_case):
    case, walks = soup_case
    sc = oracle_mod.Scene(case.V, case.F, bvh=True)
    r = oracle_mod.estimate(sc, case.rows, case.basis, walks, case.eps, case.h, exterior=False, log=True, nthreads=4)
    S, _ = oracle_mod.finalize(r["acc"], r["acc2"], case.rows.w, case.h, walks, r["discarded"])
    lt = r["log_tri"].copy()
    i = tuple(np.argwhere(r["log_status"] == oracle_mod.HIT)[3])
    lt[i] = (lt[i] + case.F.shape[0] // 2) % case.F.shape[0]
    Sr = reconstruct_from_log(oracle_mod, case, r["log_status"], lt, r["log_bary"], False)
    assert np.abs(S - Sr).max() > 1e-4 * np.abs(S).max()
