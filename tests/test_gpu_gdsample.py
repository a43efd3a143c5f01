"""GPU parity: GD sampling of transformed CNFs (tt_gd_*: every expression
simplified on the host, Table 1's operators composed over the forms on the
device, by the circuit's compiled kernel and by the interpreter) against
the oracle's float64 GD over its own forms (final logits within a float32
tolerance, hardened inputs and validity where the oracle's logit is clear of
zero), and the distinct-solution count against the distinct valid
vectors."""
import json
import pathlib

import numpy as np
import pytest

import paper_2502_08673_amd as tt
from gpu_util import note
from oracle import gdsample as G
from oracle import transform as T
from workloads import tseitin_instances

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLDEN = pathlib.Path(__file__).parent / "golden"

# float32 against float64 over five steps of rate 10: each step moves a logit
# by at most 10 |dL/dV| with dL/dV <= 2 * (number of loss terms); rounding of
# the sigmoid and the gates' products stays near 1e-6 relative, so
# 1e-3 absolute plus 1e-3 relative bounds the final logits with room.  Once
# the logits agree that closely, every logit of magnitude above 2e-3 has the
# same sign on both sides, so hardened bits are compared there.
ATOL, RTOL, CLEAR = 1e-3, 1e-3, 2e-3


def transform_on_gpu(n_vars, clauses):
    lits, coff, ioff, nv = tt.cnf_csr([(n_vars, clauses)])
    vc = torch.zeros((n_vars + 1,), dtype=torch.uint8, device="cuda")
    ex = torch.zeros((max(len(clauses), 1) * 640,), dtype=torch.uint8, device="cuda")
    ne = torch.zeros((1,), dtype=torch.int32, device="cuda")
    st = torch.zeros((1,), dtype=torch.int32, device="cuda")
    tt.cnf_transform(lits, coff, ioff, nv, vc, ex, ne, st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    recs = ex.cpu().numpy().view(tt.CNF_EXPR_DTYPE)[: int(ne.item())]
    return recs, vc.cpu().numpy()


def check(n_vars, clauses, batch, seed, compiled=True):
    """Both kernels of the sampler (the circuit's compiled kernel and the
    interpreter) against the oracle on the same logits; returns the distinct
    valid solutions found and the oracle's.  compiled=False: a circuit too
    large to compile, which only the interpreter serves."""
    recs, cls = transform_on_gpu(n_vars, clauses)
    R = T.transform(clauses)
    V0 = None
    Vo = ok = uniq = None
    got = None
    with tt.GdSampler(clauses, n_vars, recs, cls) as gd:
        assert gd.pi_vars == list(R[1])  # logit columns in the order of entry
        if compiled:
            assert gd.kernel == tt.TT_GD_COMPILED
        else:
            assert gd.kernel == tt.TT_GD_INTERPRETED
            with pytest.raises(tt.TTError) as ei:
                gd.kernel = tt.TT_GD_COMPILED
            assert ei.value.status == tt.TT_ENOTSUP
        with pytest.raises(tt.TTError) as ei:
            gd.kernel = 7
        assert ei.value.status == tt.TT_EINVAL
        V0 = np.random.default_rng(seed).normal(0, 1, (batch, gd.n_pi)).astype(np.float32)
        Vo, ok, uniq = G.sample(clauses, R, V0.astype(np.float64), lr=10.0, iters=5)
        for kernel in (tt.TT_GD_COMPILED, tt.TT_GD_INTERPRETED) if compiled else (tt.TT_GD_INTERPRETED,):
            gd.kernel = kernel
            V = torch.from_numpy(V0.copy()).cuda()
            valid = torch.zeros((batch,), dtype=torch.uint8, device="cuda")
            sol = torch.zeros((batch, gd.words), dtype=torch.int64, device="cuda")
            first = torch.zeros((batch,), dtype=torch.uint8, device="cuda")
            count = torch.zeros((1,), dtype=torch.int32, device="cuda")
            note(f"gd_sample kernel={kernel} n_vars={n_vars} clauses={len(clauses)} batch={batch}")
            gd.run(V, 10.0, 5, valid, sol)
            gd.unique(valid, sol, first, count)
            torch.cuda.synchronize()
            Vg, vg, sg = V.cpu().numpy(), valid.cpu().numpy().astype(bool), sol.cpu().numpy().view(np.uint64)
            assert np.allclose(Vg, Vo, atol=ATOL, rtol=RTOL), kernel
            clear = (np.abs(Vo) > CLEAR).all(axis=1)
            assert clear.mean() > 0.9
            assert np.array_equal((Vg[clear] > 0), (Vo[clear] > 0)), kernel
            assert np.array_equal(vg[clear], ok[clear]), kernel
            # hardened bits of the solution words are the signs of the final logits
            for q in range(gd.n_pi):
                bit = (sg[:, q // 64] >> np.uint64(q % 64)) & np.uint64(1)
                assert np.array_equal(bit.astype(bool), Vg[:, q] > 0), kernel
            # distinct valid solutions: one first sample each, count = distinct vectors
            f = first.cpu().numpy().astype(bool)
            distinct = {tuple(sg[i]) for i in np.nonzero(vg)[0]}
            assert int(count.item()) == len(distinct) == f.sum(), kernel
            assert {tuple(sg[i]) for i in np.nonzero(f)[0]} == distinct and not (f & ~vg).any(), kernel
            got = len(distinct) if got is None else got
    return got, len(uniq)


def test_fig1_cnf_samples():
    g = json.loads((GOLDEN / "fig1_cnf.json").read_text())
    got, want = check(14, T.parse_dimacs(g["dimacs"]), batch=1000, seed=0)
    assert got == want == 32


@pytest.mark.parametrize("k", [0, 1, 2])
def test_random_tseitin_instances(k):
    n_vars, clauses = tseitin_instances(seed=300 + k, n_inst=1, n_gates=(20, 40))[0]
    check(n_vars, clauses, batch=777, seed=k)


def test_large_form_temporaries_in_the_global_block():
    """x10 = exactly one of x1 .. x9 (a clause per pair, one per input, one
    for at least one): its minimal SOP is the nine minterms, 80 gates, so the
    form's 79 temporaries need 40 KiB per wave and stay in the global block
    beside the variables (forms with fewer temporaries keep them in LDS);
    then x10 OR x11 and x11 -> x12 as an auxiliary output."""
    n = 9
    f = n + 1
    C = [[-f] + list(range(1, n + 1))]
    C += [[-f, -i, -j] for i in range(1, n + 1) for j in range(i + 1, n + 1)]
    C += [[f, -i] + [j for j in range(1, n + 1) if j != i] for i in range(1, n + 1)]
    C += [[f, 11], [-11, 12]]
    R = T.transform(C)
    form = G.simplify(R[3][0])

    def gates(t):
        return 0 if t[0] in ("VAR", "CONST") else (t[0] != "NOT") + sum(gates(u) for u in t[1:])

    assert R[3][0].out == f and G.form_vars(form) == set(range(1, n + 1)) and gates(form) == 80
    check(12, C, batch=300, seed=7)


def test_constant_and_auxiliary_outputs_on_primary_inputs():
    """Fig. 1 plus a unit clause on the primary input x1 (an auxiliary
    output on a primary input) and x15 = 0 followed by x16 = not x15 (x15
    becomes both a constant output and a primary input: a (P - 0)^2 loss
    term)."""
    g = json.loads((GOLDEN / "fig1_cnf.json").read_text())
    clauses = T.parse_dimacs(g["dimacs"]) + [[1], [-15], [15, 16], [-15, -16]]
    PO, PI, IV, E = T.transform(clauses)
    assert 15 in PO and 15 in PI and 1 in PI and any(e.kind == "AUX" and e.vars == [1] for e in E)
    check(16, clauses, batch=500, seed=5)


def test_large_circuit_uses_global_state():
    """A 200-gate circuit (over 128 variables in use): the state leaves LDS
    for a global workspace; same results as the oracle."""
    n_vars, clauses = tseitin_instances(seed=400, n_inst=1, n_in=(30, 30), n_gates=(200, 200), window=48)[0]
    assert n_vars > 200
    check(n_vars, clauses, batch=300, seed=9)


@pytest.mark.parametrize("batch,iters,lr", [(1, 5, 10.0), (257, 5, 10.0), (300, 0, 10.0), (300, 3, 0.5)])
def test_batch_edges_iterations_and_rate(batch, iters, lr):
    """One sample, a partial block of 256 threads, no GD step (hardening of
    the initial logits only) and another rate and step count: both kernels
    against the oracle, logits, validity and solution bits."""
    n_vars, clauses = tseitin_instances(seed=305, n_inst=1, n_gates=(20, 40))[0]
    recs, cls = transform_on_gpu(n_vars, clauses)
    R = T.transform(clauses)
    with tt.GdSampler(clauses, n_vars, recs, cls) as gd:
        V0 = np.random.default_rng(batch + iters).normal(0, 1, (batch, gd.n_pi)).astype(np.float32)
        Vo, ok, _ = G.sample(clauses, R, V0.astype(np.float64), lr=lr, iters=iters)
        for kernel in (tt.TT_GD_COMPILED, tt.TT_GD_INTERPRETED):
            gd.kernel = kernel
            V = torch.from_numpy(V0.copy()).cuda()
            valid = torch.full((batch,), 7, dtype=torch.uint8, device="cuda")
            sol = torch.zeros((batch, gd.words), dtype=torch.int64, device="cuda")
            note(f"gd_sample kernel={kernel} batch={batch} iters={iters} lr={lr}")
            gd.run(V, lr, iters, valid, sol)
            torch.cuda.synchronize()
            Vg, vg = V.cpu().numpy(), valid.cpu().numpy()
            assert np.allclose(Vg, Vo, atol=ATOL, rtol=RTOL), kernel
            assert set(np.unique(vg)) <= {0, 1}, kernel
            clear = (np.abs(Vo) > CLEAR).all(axis=1)
            assert np.array_equal(vg[clear].astype(bool), ok[clear]), kernel
            sg = sol.cpu().numpy().view(np.uint64)
            for q in range(gd.n_pi):
                bit = (sg[:, q // 64] >> np.uint64(q % 64)) & np.uint64(1)
                assert np.array_equal(bit.astype(bool), Vg[:, q] > 0), kernel


@pytest.mark.parametrize("big", [False, True])
def test_run_from_matches_in_place(big):
    """tt_gd_run_from on both kernels: with the final logits not kept (null)
    or written to a buffer of their own, the valid flags and solution words
    equal the in-place run's bit for bit, the logits written apart equal the
    in-place final logits, and the initial logits are left unchanged.  The
    large circuit takes the interpreter's global-state form."""
    if big:
        n_vars, clauses = tseitin_instances(seed=400, n_inst=1, n_in=(30, 30), n_gates=(200, 200), window=48)[0]
    else:
        n_vars, clauses = tseitin_instances(seed=306, n_inst=1, n_gates=(20, 40))[0]
    recs, cls = transform_on_gpu(n_vars, clauses)
    batch = 300
    with tt.GdSampler(clauses, n_vars, recs, cls) as gd:
        V0h = np.random.default_rng(41).normal(0, 1, (batch, gd.n_pi)).astype(np.float32)
        for kernel in (tt.TT_GD_COMPILED, tt.TT_GD_INTERPRETED):
            gd.kernel = kernel
            outs = {}
            for mode in ("in_place", "apart", "none"):
                V0 = torch.from_numpy(V0h.copy()).cuda()
                V = torch.full_like(V0, 7.0) if mode == "apart" else None
                valid = torch.full((batch,), 9, dtype=torch.uint8, device="cuda")
                sol = torch.zeros((batch, gd.words), dtype=torch.int64, device="cuda")
                note(f"gd run_from kernel={kernel} mode={mode} n_vars={n_vars} batch={batch}")
                if mode == "in_place":
                    gd.run(V0, 10.0, 5, valid, sol)
                else:
                    gd.run_from(V0, V, 10.0, 5, valid, sol)
                torch.cuda.synchronize()
                outs[mode] = (V0.cpu().numpy(), None if V is None else V.cpu().numpy(), valid.cpu().numpy(),
                              sol.cpu().numpy())
            final, _, v_ip, s_ip = outs["in_place"]
            for mode in ("apart", "none"):
                v0, _, v, sol_ = outs[mode]
                assert np.array_equal(v, v_ip) and np.array_equal(sol_, s_ip), (kernel, mode)
                assert np.array_equal(v0, V0h), (kernel, mode)
            assert np.array_equal(outs["apart"][1], final), kernel
            assert not np.array_equal(final, V0h), kernel
        # no initial logits: refused before any device work
        valid = torch.zeros((batch,), dtype=torch.uint8, device="cuda")
        sol = torch.zeros((batch, gd.words), dtype=torch.int64, device="cuda")
        assert tt.lib().tt_gd_run_from(gd._h, None, None, batch, 10.0, 5, valid.data_ptr(), sol.data_ptr(),
                                       None) == tt.TT_EINVAL


@pytest.mark.parametrize("big", [False, True])
def test_sample_unique_matches_run_then_unique(big):
    """tt_gd_sample_unique on both kernels against tt_gd_run_from followed by
    tt_gd_unique: the same valid flags, solution words and count (added to a
    count that is not zero); the samples marked first are valid and mark
    each distinct valid solution once (which sample is marked may differ).
    300 samples: the compiled kernel's 512 threads clear the filter's
    1024-place table in a stride loop."""
    if big:
        n_vars, clauses = tseitin_instances(seed=400, n_inst=1, n_in=(30, 30), n_gates=(200, 200), window=48)[0]
    else:
        n_vars, clauses = tseitin_instances(seed=307, n_inst=1, n_gates=(20, 40))[0]
    recs, cls = transform_on_gpu(n_vars, clauses)
    batch = 300
    with tt.GdSampler(clauses, n_vars, recs, cls) as gd:
        V0 = torch.from_numpy(np.random.default_rng(43).normal(0, 1, (batch, gd.n_pi)).astype(np.float32)).cuda()
        for kernel in (tt.TT_GD_COMPILED, tt.TT_GD_INTERPRETED):
            gd.kernel = kernel
            res = []
            for fused in (False, True):
                valid = torch.full((batch,), 9, dtype=torch.uint8, device="cuda")
                sol = torch.zeros((batch, gd.words), dtype=torch.int64, device="cuda")
                first = torch.full((batch,), 9, dtype=torch.uint8, device="cuda")
                count = torch.full((1,), 5, dtype=torch.int32, device="cuda")
                note(f"gd sample_unique kernel={kernel} fused={fused} n_vars={n_vars} batch={batch}")
                if fused:
                    gd.sample_unique(V0, None, 10.0, 5, valid, sol, first, count)
                else:
                    gd.run_from(V0, None, 10.0, 5, valid, sol)
                    gd.unique(valid, sol, first, count)
                torch.cuda.synchronize()
                res.append((valid.cpu().numpy().astype(bool), sol.cpu().numpy().view(np.uint64),
                            first.cpu().numpy(), int(count.item())))
            (v1, s1, _, c1), (v2, s2, f2, c2) = res
            assert np.array_equal(v1, v2) and np.array_equal(s1, s2), kernel
            distinct = {tuple(s1[i]) for i in np.nonzero(v1)[0]}
            assert c1 == c2 == 5 + len(distinct) and len(distinct) > 1, kernel
            assert set(np.unique(f2)) <= {0, 1}, kernel
            marked = [tuple(s2[i]) for i in np.nonzero(f2)[0]]
            assert len(marked) == len(set(marked)) and set(marked) == distinct, kernel
            assert not (f2.astype(bool) & ~v2).any(), kernel


def test_benchmark_circuit_full_batch():
    """The benchmark's launch: its 36-input circuit (a 60-gate Tseitin
    circuit, last output forced) transformed on the device, 2^20 samples
    through tt_gd_sample_unique with the compiled kernel.  The count equals
    the number of distinct valid solution vectors of the whole batch (counted
    on the host), each marked once; every 64th sample's validity and
    solution bits match the oracle's where its final logits are clear of
    zero."""
    n_vars, clauses = tseitin_instances(20250212 + 301, 1, n_in=(48, 48), n_gates=(60, 60), window=64)[0]
    recs, cls = transform_on_gpu(n_vars, clauses)
    R = T.transform(clauses)
    B = 1 << 20
    with tt.GdSampler(clauses, n_vars, recs, cls) as gd:
        assert gd.kernel == tt.TT_GD_COMPILED
        V0h = np.random.default_rng(47).normal(0, 1, (B, gd.n_pi)).astype(np.float32)
        V0 = torch.from_numpy(V0h).cuda()
        valid = torch.empty((B,), dtype=torch.uint8, device="cuda")
        sol = torch.empty((B, gd.words), dtype=torch.int64, device="cuda")
        first = torch.empty((B,), dtype=torch.uint8, device="cuda")
        count = torch.zeros((1,), dtype=torch.int32, device="cuda")
        note(f"gd benchmark circuit n_pi={gd.n_pi} batch={B}")
        gd.sample_unique(V0, None, 10.0, 5, valid, sol, first, count)
        torch.cuda.synchronize()
        vg = valid.cpu().numpy().astype(bool)
        sg = sol.cpu().numpy().view(np.uint64)
        f = first.cpu().numpy().astype(bool)
    distinct = np.unique(sg[vg], axis=0)
    assert int(count.item()) == len(distinct) == f.sum() and not (f & ~vg).any()
    assert len(np.unique(sg[f], axis=0)) == len(distinct)
    rows = np.arange(0, B, 64)
    Vo, ok, _ = G.sample(clauses, R, V0h[rows].astype(np.float64), lr=10.0, iters=5)
    clear = (np.abs(Vo) > CLEAR).all(axis=1)
    assert clear.mean() > 0.9
    assert np.array_equal(vg[rows][clear], ok[clear])
    for q in range(Vo.shape[1]):
        bit = (sg[rows, q // 64] >> np.uint64(q % 64)) & np.uint64(1)
        assert np.array_equal(bit.astype(bool)[clear], Vo[clear, q] > 0)


def test_unique_two_word_solutions():
    """tt_gd_unique on solutions of two words (80 primary inputs: 40
    independent two-literal clauses), on buffers built here: rows drawn from
    a few thousand first and second words, so the batch holds repeats, rows
    equal in the first word only and rows equal in the second word only,
    with one row in ten invalid; a batch of five passes of the filter's grid
    and a ragged tail.  Count and marks against the distinct valid rows
    counted on the host."""
    clauses = [[2 * k + 1, 2 * k + 2] for k in range(40)]
    recs, cls = transform_on_gpu(80, clauses)
    with tt.GdSampler(clauses, 80, recs, cls) as gd:
        assert gd.n_pi == 80 and gd.words == 2
        rng = np.random.default_rng(11)
        B = 5 * 262144 + 7
        w0 = rng.integers(0, 2**63, size=4000, dtype=np.int64)
        w1 = rng.integers(0, 2**63, size=3000, dtype=np.int64)
        rows = np.stack([w0[rng.integers(0, 4000, B)], w1[rng.integers(0, 3000, B)]], axis=1)
        vh = (rng.random(B) < 0.9).astype(np.uint8)
        valid = torch.from_numpy(vh).cuda()
        sol = torch.from_numpy(rows).cuda()
        first = torch.full((B,), 7, dtype=torch.uint8, device="cuda")
        count = torch.zeros((1,), dtype=torch.int32, device="cuda")
        note(f"gd unique two words batch={B}")
        gd.unique(valid, sol, first, count)
        torch.cuda.synchronize()
        f = first.cpu().numpy()
    assert set(np.unique(f)) <= {0, 1}
    f = f.astype(bool)
    v = vh.astype(bool)
    distinct = np.unique(rows[v], axis=0)
    assert len(distinct) > 100000  # the rows repeat, and not only in one word
    assert int(count.item()) == len(distinct) == f.sum() and not (f & ~v).any()
    assert np.array_equal(np.unique(rows[f], axis=0), distinct)


def test_circuit_too_large_to_compile_uses_the_interpreter():
    """Over 512 variables in use: no compiled kernel (selecting it is
    TT_ENOTSUP), the interpreter matches the oracle."""
    n_vars, clauses = tseitin_instances(seed=401, n_inst=1, n_in=(40, 40), n_gates=(560, 560), window=48)[0]
    assert n_vars > 560
    check(n_vars, clauses, batch=200, seed=11, compiled=False)


def test_wide_expressions():
    """An AND of eight inputs and an OR of seven (forms: an AND chain of
    eight literals, an OR chain of seven), their XOR forced to 1."""
    ins_a, ins_b = list(range(1, 9)), list(range(10, 17))
    cl = [[9] + [-x for x in ins_a]] + [[-9, x] for x in ins_a]          # x9 = AND(x1..x8)
    cl += [[-17] + ins_b] + [[17, -x] for x in ins_b]                   # x17 = OR(x10..x16)
    cl += [[-9, -17, -18], [9, 17, -18], [9, -17, 18], [-9, 17, 18]]    # x18 = x9 XOR x17
    cl += [[18]]
    PO, PI, IV, E = T.transform(cl)
    assert max(len(e.vars) for e in E) == 8
    check(18, cl, batch=400, seed=13)



def test_reconvergent_forms():
    """Expressions whose forms read a variable more than once: a majority of
    three (ab + ac + bc) and a multiplexer feeding a three-input parity
    (an XOR chain), the parity constrained to 1; the composed gates differ
    from the tables' exact probabilities here, so this pins the composition."""
    cl = [[-4, 1, 2], [-4, 1, 3], [-4, 2, 3], [4, -1, -2], [4, -1, -3], [4, -2, -3]]   # x4 = MAJ(x1, x2, x3)
    cl += [[-7, -5, 4], [-7, 5, 6], [7, -5, -4], [7, 5, -6]]                          # x7 = x5 ? x4 : x6
    cl += [[-9, 7, 8, 1], [-9, 7, -8, -1], [-9, -7, 8, -1], [-9, -7, -8, 1],
           [9, -7, -8, -1], [9, -7, 8, 1], [9, 7, -8, 1], [9, 7, 8, -1]]              # x9 = x7 ^ x8 ^ x1
    cl += [[9]]
    PO, PI, IV, E = T.transform(cl)
    assert 4 in IV and 7 in IV
    check(9, cl, batch=600, seed=17)
