"""GPU edge cases through the C ABI: non-convergence, zero load, several
right-hand sides, reproducibility, symmetry and argument checks."""

import ctypes

import numpy as np
import pytest

import synth
from gpu_common import cuda_vec

pytestmark = pytest.mark.gpu


def _solver(prob):
    import paper_0911_5730_amd as P
    return P.Solver(prob)


def test_maxit_reports_noconv_with_last_iterate():
    import paper_0911_5730_amd as P
    prob = synth.square_problem(32, 4, constraints="corners", kmode="loguniform", kmax_exp=3, seed=31)
    with _solver(prob) as S:
        f = cuda_vec(prob.f[0])
        with pytest.raises(P.BDDCError) as ei:
            S.solve(f, maxit=2)
        assert ei.value.name == "BDDC_ENOCONV"
        u, it, rr = S.solve(f, maxit=2, allow_noconv=True)
        assert it == [2] and rr[0] > 1e-8
        assert np.isfinite(u.cpu().numpy()).all()


def test_zero_load_gives_zero_solution():
    prob = synth.square_problem(16, 4, constraints="corners_edges", seed=32)
    with _solver(prob) as S:
        u, it, rr = S.solve(cuda_vec(np.zeros(prob.n_free)))
        assert it == [0] and rr == [0.0]
        assert not u.cpu().numpy().any()


def test_several_rhs_equal_separate_solves_bitwise():
    import torch
    prob = synth.square_problem(48, 4, levels=3, groups=(2, 2), constraints="adaptive", tau=3.0,
                                kmode="loguniform", kmax_exp=3, nrhs=3, seed=33)
    with _solver(prob) as S:
        F = cuda_vec(prob.f)
        U, its, rrs = S.solve(F)
        for c in range(3):
            u, it, rr = S.solve(F[c].contiguous())
            assert it[0] == its[c]
            assert torch.equal(u, U[c])


def test_repeated_setup_and_solve_are_bitwise_reproducible():
    import torch
    prob = synth.square_problem(64, 8, levels=3, groups=(2, 2), constraints="adaptive", tau=2.0,
                                kmode="loguniform", kmax_exp=4, channels=2, seed=34)
    f = cuda_vec(prob.f[0])
    outs = []
    for _ in range(2):
        with _solver(prob) as S:
            outs.append(S.solve(f)[0])
    assert torch.equal(outs[0], outs[1])


def test_preconditioner_is_symmetric():
    prob = synth.square_problem(48, 6, levels=3, groups=(3, 3), constraints="adaptive", tau=2.0,
                                kmode="loguniform", kmax_exp=5, channels=2, seed=35)
    rng = np.random.default_rng(0)
    r, s = rng.standard_normal((2, prob.n_free))
    with _solver(prob) as S:
        Mr = S.apply(cuda_vec(r)).cpu().numpy()
        Ms = S.apply(cuda_vec(s)).cpu().numpy()
    a, b = s @ Mr, r @ Ms
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def test_smallest_mesh():
    prob = synth.square_problem(2, 1, seed=36)          # one free node
    with _solver(prob) as S:
        u, it, rr = S.solve(cuda_vec(prob.f[0]))
        assert abs(u.cpu().numpy()[0] - prob.f[0][0] / (8.0 / 3.0)) < 1e-14


def test_device_argument_validation():
    import paper_0911_5730_amd as P
    prob = synth.config(1)
    with _solver(prob) as S:
        lib = S.lib
        r = cuda_vec(np.ones(prob.n_free))
        z = cuda_vec(np.zeros(prob.n_free))
        st = lib.bddc_apply(S.h, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(z.data_ptr()), 1,
                            prob.n_free - 1, None)
        assert st == -1
        st = lib.bddc_apply(S.h, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(r.data_ptr()), 1,
                            prob.n_free, None)
        assert st == -1
        iters = (ctypes.c_int32 * 1)()
        rel = (ctypes.c_double * 1)()
        st = lib.bddc_solve(S.h, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(z.data_ptr()), 1,
                            prob.n_free, -1.0, 10, iters, rel, None)
        assert st == -1
        with pytest.raises(P.BDDCError):
            S.edge_eigs(1, 0)                            # not an adaptive set-up
        assert lib.bddc_query(None, None) == -1
    lib.bddc_destroy(None)


def test_concurrent_handles_on_two_streams_match_alone():
    """Independent problems set up and solved from two host threads, each with
    its own stream and handles, interleave on the device; every result must
    equal (bitwise) the same problem solved alone."""
    import threading

    import torch

    import paper_0911_5730_amd as P
    from test_gpu_parity import _case

    probs = [_case("adaptive3"), _case("corners_kjump")]
    alone = []
    for prob in probs:
        S = P.Solver(prob)
        try:
            u, it, _ = S.solve(cuda_vec(prob.f[0]))
            alone.append((u.cpu().numpy(), int(it[0])))
        finally:
            S.close()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    results = [[], []]
    errors = []

    def worker(k):
        try:
            prob = probs[k]
            f = cuda_vec(prob.f[0])
            torch.cuda.synchronize()
            for _ in range(3):
                S = P.Solver(prob, stream=streams[k])
                try:
                    u, it, _ = S.solve(f, stream=streams[k])
                    torch.cuda.synchronize()
                    results[k].append((u.cpu().numpy(), int(it[0])))
                finally:
                    S.close()
        except Exception as e:
            errors.append(e)

    th = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    for k in range(2):
        assert len(results[k]) == 3
        for u, it in results[k]:
            assert it == alone[k][1]
            assert np.array_equal(u, alone[k][0])


def test_serving_loop_results_alone_equal_in_the_mix():
    """Requests of different sizes admitted onto two concurrent slots: every
    solution equals (bitwise) the same request solved alone; with an HBM
    budget below two requests' footprint only one is admitted at a time."""
    import synth
    from paper_0911_5730_amd.serve import Request, Server

    import paper_0911_5730_amd as P

    stream = synth.request_stream(6, seed=77)
    alone = []
    for _, prob in stream:
        S = P.Solver(prob, precision="fp32")
        try:
            u, it, _ = S.solve(cuda_vec(prob.f).reshape(prob.f.shape))
            alone.append((u.cpu().numpy(), it))
        finally:
            S.close()
    for budget, limit in ((None, 2), (1, 1)):
        srv = Server(slots=2, hbm_budget=budget)
        try:
            reqs = [srv.submit(Request(prob=p, rhs=p.f, precision="fp32")) for _, p in stream]
            srv.drain()
        finally:
            srv.close()
        assert srv.max_active <= limit
        for r, (u, it) in zip(reqs, alone):
            assert r.error is None, r.error
            assert r.iterations == it
            assert np.array_equal(r.solution, u)
        st = srv.stats()
        assert st["requests"] == len(stream) and st["latency_ms"]["p99"] >= st["latency_ms"]["p50"]


def test_stepwise_solve_matches_solve_and_guards_the_handle():
    """bddc_solve_begin / _advance / _poll / _end give bitwise the solution and
    iteration counts of bddc_solve (the same launches, in chunks); while a
    stepwise solve is in progress the handle refuses other solves and applies
    with BDDC_EBUSY, and works normally after the end."""
    import time

    import torch

    import paper_0911_5730_amd as P
    prob = synth.square_problem(48, 4, levels=3, groups=(2, 2), constraints="adaptive", tau=3.0,
                                kmode="loguniform", kmax_exp=3, nrhs=3, seed=33)
    with _solver(prob) as S:
        F = cuda_vec(prob.f)
        U, its, rr = S.solve(F)
        S.begin(F)
        with pytest.raises(P.BDDCError) as ei:
            S.solve(F)
        assert ei.value.name == "BDDC_EBUSY"
        with pytest.raises(P.BDDCError) as ei:
            S.apply(F[0].contiguous())
        assert ei.value.name == "BDDC_EBUSY"
        states = []
        S.advance(4)
        for _ in range(1000):
            st = S.poll()
            states.append(st)
            if st == 1:
                break
            if st == 0:
                S.advance(4)
            else:
                time.sleep(1e-4)
        assert states[-1] == 1
        U2, its2, rr2 = S.end()
        assert its2 == its and rr2 == rr
        assert torch.equal(U2, U)
        U3, its3, _ = S.solve(F)
        assert its3 == its and torch.equal(U3, U)


def test_serving_admits_requests_while_others_run():
    """Continuous batching: a request that arrives while a long solve is in
    flight is set up and started at an iteration boundary of the running
    solve (both in flight together); both results equal their solves alone
    (bitwise)."""
    import time

    import paper_0911_5730_amd as P
    from paper_0911_5730_amd.serve import Request, Server
    big = synth.square_problem(1024, 64, levels=3, groups=(4, 4), constraints="adaptive", tau=10.0,
                               kmode="one", nrhs=8, seed=61)
    small = synth.square_problem(64, 8, constraints="adaptive", tau=10.0, kmode="loguniform", kmax_exp=2,
                                 nrhs=1, seed=62)
    alone = []
    for prob in (big, small):
        S = P.Solver(prob, precision="fp32")
        try:
            u, it, _ = S.solve(cuda_vec(prob.f), rtol=1e-10)
            alone.append((u.cpu().numpy(), it))
        finally:
            S.close()
    srv = Server(slots=4, chunk=2)
    try:
        rb = srv.submit(Request(prob=big, rhs=big.f, precision="fp32", rtol=1e-10))
        while not rb.started:
            time.sleep(1e-3)
        rs = srv.submit(Request(prob=small, rhs=small.f, precision="fp32", rtol=1e-10))
        srv.drain()
    finally:
        srv.close()
    assert rb.error is None and rs.error is None, (rb.error, rs.error)
    print(f"big: started {rb.started:.4f} done {rb.done:.4f}; small: arrival {rs.arrival:.4f} started "
          f"{rs.started:.4f} done {rs.done:.4f}", flush=True)
    assert rs.started < rb.done
    assert srv.max_active >= 2
    for r, (u, it) in zip((rb, rs), alone):
        assert r.iterations == it
        assert np.array_equal(r.solution, u)


def test_serving_resident_problems_merge_loads_and_match_alone():
    """Requests against a few shared problems: a resident problem is reused
    without a new set-up and the pending loads of one problem are merged into
    one blocked solve; every request's solution equals (bitwise) the request
    solved alone on a fresh set-up."""
    import synth
    from paper_0911_5730_amd.serve import Request, Server

    import paper_0911_5730_amd as P

    stream = synth.request_stream(12, seed=78, problems=3, sides=(64, 128), hh=(8, 16))
    alone = []
    for _, prob in stream:
        S = P.Solver(prob, precision="fp32")
        try:
            u, it, _ = S.solve(cuda_vec(prob.f).reshape(prob.f.shape))
            alone.append((u.cpu().numpy(), it))
        finally:
            S.close()
    srv = Server(slots=2, resident=True)
    try:
        # all submitted at once, so loads of one problem can merge
        reqs = [srv.submit(Request(prob=p, rhs=p.f, precision="fp32", key=p.meta["problem"])) for _, p in stream]
        srv.drain()
        st = srv.stats()
    finally:
        srv.close()
    for r, (u, it) in zip(reqs, alone):
        assert r.error is None, r.error
        assert r.iterations == it
        assert np.array_equal(r.solution, u)
    print(f"serving resident: {st}", flush=True)
    assert st["reused"] > 0 and st["mean_batch"] > 1.0


def test_disconnected_coarse_substructure_is_rejected():
    """A level-2 substructure made of two level-1 substructures that share
    no coarse dof would carry a null space per piece: set-up refuses it with
    BDDC_EPARTITION instead of meeting a singular pivot."""
    import paper_0911_5730_amd as P
    prob = synth.square_problem(16, 4, levels=3, groups=(2, 2), kmode="loguniform", kmax_exp=1, seed=37)
    agg = np.ones(16, dtype=np.int32)
    agg[0] = agg[15] = 0                     # opposite corners of the 4 x 4 partition
    prob.agglom = [agg]
    with pytest.raises(P.BDDCError) as ei:
        P.Solver(prob)
    assert ei.value.name == "BDDC_EPARTITION"


def test_bf16_form_refused_where_its_factor_does_not_fit_lds():
    """The factored BF16 form stages each substructure's W in LDS: with a
    centre substructure of 256 interface dofs (3 x 3 substructures of 64 x 64
    elements) the set-up refuses it with BDDC_EUNSUPPORTED, while the FP32
    form of the same problem sets up and solves."""
    import paper_0911_5730_amd as P
    prob = synth.square_problem(192, 3, kmode="one", seed=41)
    print("bf16 refusal: 192 x 192, 3 x 3 substructures", flush=True)
    with pytest.raises(P.BDDCError) as ei:
        P.Solver(prob, precision="bf16")
    assert ei.value.name == "BDDC_EUNSUPPORTED"
    with P.Solver(prob, precision="fp32") as S:
        _, it, rr = S.solve(cuda_vec(prob.f[0]))
        assert rr[0] <= 1e-8 and it[0] > 0
