"""Launch configuration and its autotuner (bddc_get_tuning / bddc_set_tuning /
bddc_autotune).

The knobs change how the same method is launched, not what it computes: the
partial-sum mode, graph replay and the number of PCG iterations between host
checks leave the iterates bitwise unchanged; the deep-level paths agree with
the oracle.  The autotuner installs the fastest configuration it measured and
remembers it for the problem's shape, so a later set-up of that shape starts
from it.
"""

import numpy as np
import pytest

from gpu_common import check_solution, cuda_vec, run_pair
from test_gpu_parity import _case

pytestmark = pytest.mark.gpu


def test_knobs_leave_iterates_bitwise_and_paths_match_oracle():
    import torch

    import paper_0911_5730_amd as P
    prob = _case("adaptive3")
    f = cuda_vec(prob.f[0])
    with P.Solver(prob) as S:
        t0 = S.tuning()
        assert set(t0["available"]) >= {"coop", "wide", "levels"}, t0
        u0, it0, _ = S.solve(f, rtol=1e-10)
        for knob, vals in (("finalize", (0, 1, 2, 3)), ("graph", (0, 1)), ("check", (4, 8, 16))):
            for v in vals:
                print(f"tuning {knob}={v}", flush=True)
                S.set_tuning(**{knob: v})
                for _ in range(2):   # with a graph: capture, then replay
                    u, it, _ = S.solve(f, rtol=1e-10)
                    assert it == it0 and torch.equal(u, u0), (knob, v)
            S.set_tuning(**{knob: t0[knob]})
    for path in ("wide", "levels"):
        print(f"tuning deep_path={path}", flush=True)
        S, B, ug, it, rr, o = run_pair(prob, tuning={"deep_path": path})
        try:
            assert S.tuning()["deep_path"] == path
            assert abs(it - o["iters"]) <= 1
            check_solution(S, B, ug, o)
        finally:
            S.close()


def test_autotune_installs_and_remembers_the_fastest():
    import paper_0911_5730_amd as P
    prob = _case("adaptive3_h16")
    F = cuda_vec(prob.f)
    with P.Solver(prob) as S:
        t = S.autotune(F, reps=2)
        print(f"autotune: {t}", flush=True)
        assert t["deep_path"] in t["available"]
        assert t["finalize"] in (0, 1, 2, 3) and t["graph"] in (0, 1) and t["check"] in (4, 8, 16)
        assert t["solve_ms"] > 0
        assert S.tuning() == t
    # a new set-up of the same shape starts from the remembered choice
    S, B, ug, it, rr, o = run_pair(prob)
    try:
        assert S.tuning() == t
        assert abs(it - o["iters"]) <= 1
        check_solution(S, B, ug, o)
    finally:
        S.close()


def test_set_tuning_rejects_what_the_setup_cannot_run():
    import paper_0911_5730_amd as P
    prob = _case("corners_kjump")          # two levels: the coarse problem is solved directly
    with P.Solver(prob) as S:
        assert S.tuning()["available"] == ["levels"]
        for bad in ({"deep_path": "coop"}, {"check": 5}, {"finalize": 4}, {"graph": -1}):
            with pytest.raises(P.BDDCError) as ei:
                S.set_tuning(**bad)
            assert ei.value.name == "BDDC_EINVAL"
        u, it, rr = S.solve(cuda_vec(prob.f[0]))
        assert np.isfinite(u.cpu().numpy()).all() and rr[0] <= 1e-8


def test_row_block_launches_take_finalize_1_only(monkeypatch):
    """The row-block launches of wide interfaces read the summed scalars of
    the one-block sums: the other forms are refused, and the solve still runs."""
    import paper_0911_5730_amd as P
    prob = _case("adaptive3")
    # a choice remembered for this shape without row blocks is not taken by a
    # set-up that plans them
    with P.Solver(prob) as S:
        S.autotune(cuda_vec(prob.f[:1]), reps=1)
    monkeypatch.setenv("BDDC_PCG_ROWS", "1")
    monkeypatch.setenv("BDDC_PCG_FINALIZE", "2")   # (taken as 1 with row blocks)
    with P.Solver(prob) as S:
        assert S.tuning()["finalize"] == 1
        for fin in (0, 2, 3):
            with pytest.raises(P.BDDCError) as ei:
                S.set_tuning(finalize=fin)
            assert ei.value.name == "BDDC_EINVAL"
        u, it, rr = S.solve(cuda_vec(prob.f[0]))
        assert np.isfinite(u.cpu().numpy()).all() and rr[0] <= 1e-8
