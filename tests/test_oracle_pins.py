"""Pins of the CPU oracle against facts that do not come from the oracle itself:
dense brute force, closed forms, invariants and library routines."""
import numpy as np
import pytest

from oracle import brute as bf
from oracle import mpo_oracle as mo
from paper_2604_21908_amd import circuitgen as cg

X = np.array([[0, 1], [1, 0]], dtype=np.complex128)


def peak_operator(c):
    """X^b K as a dense matrix, from the generator's undressed K gates."""
    k = bf.circuit_unitary(c.n, c.k_gates)
    xb = np.array([[1.0 + 0j]])
    for q in range(c.n):
        xb = np.kron(xb, X if c.peak[q] else np.eye(2))
    return xb @ k


# ------------------------------------------------------------------ inputs
@pytest.mark.parametrize("reading", ["A", "B"])
@pytest.mark.parametrize("n,depth,seed", [(6, 3, 1), (7, 4, 2), (8, 4, 3)])
def test_generator_operator_is_planted_peak(reading, n, depth, seed):
    c = cg.mirrored_peaked_circuit(n, depth, seed, reading=reading)
    for q0, q1, u in c.gates:
        assert q1 == q0 + 1
        assert np.allclose(u.conj().T @ u, np.eye(4), atol=1e-12)
    assert np.allclose(bf.circuit_unitary(n, c.gates), peak_operator(c), atol=1e-11)


def test_generator_seeded_and_obfuscated():
    a = cg.mirrored_peaked_circuit(10, 4, 7)
    b = cg.mirrored_peaked_circuit(10, 4, 7)
    c = cg.mirrored_peaked_circuit(10, 4, 8)
    assert a.digest() == b.digest() and a.digest() != c.digest()
    # no gate is a bare SWAP and no two consecutive gates on a pair cancel literally
    for q0, q1, u in a.gates:
        assert not np.allclose(np.abs(u), np.abs(mo.SWAP4))
    for (p0, p1, u), (r0, r1, v) in zip(a.gates, a.gates[1:]):
        if (p0, p1) == (r0, r1):
            assert not np.allclose(v @ u, np.eye(4) * (v @ u)[0, 0], atol=1e-6)


def test_oets_sorts_and_inverse_cancels():
    rng = np.random.default_rng(0)
    for n in (2, 5, 9, 16):
        perm = rng.permutation(n)
        a = list(perm)
        for rnd in cg.oets_swaps(perm):
            for i, j in rnd:
                a[i], a[j] = a[j], a[i]
        assert a == sorted(a)


# ----------------------------------------------------------- truncation rule
def brute_rank(s, chi_max, cutoff, mode):
    s = np.asarray(s)
    if mode == "rel_sv":
        k = sum(1 for x in s if x > cutoff * s[0])
    else:
        tot = sum(x * x for x in s)
        k = next(kk for kk in range(len(s) + 1) if sum(x * x for x in s[kk:]) <= cutoff * tot)
    return max(1, min(k, chi_max, len(s)))


def test_truncation_rank_hand_spectra():
    assert mo.truncation_rank([1.0, 0.5, 1e-13], 10, 1e-12, "rel_sv") == 2
    assert mo.truncation_rank(np.sqrt([0.9, 0.09, 0.009, 0.001]), 10, 0.002, "weight") == 3
    assert mo.truncation_rank(np.sqrt([0.9, 0.09, 0.009, 0.001]), 2, 0.002, "weight") == 2
    assert mo.truncation_rank(np.sqrt([0.9, 0.09, 0.009, 0.001]), 10, 0.0, "weight") == 4
    assert mo.truncation_rank([1.0, 0.0, 0.0], 10, 1e-12, "weight") == 1
    assert mo.truncation_rank([0.0, 0.0], 10, 1e-12, "rel_sv") == 1


def test_truncation_rank_matches_brute_force_and_is_monotone():
    rng = np.random.default_rng(1)
    for _ in range(300):
        s = np.sort(rng.exponential(size=rng.integers(1, 30)) ** 4)[::-1]
        for mode in ("rel_sv", "weight"):
            cut = 10.0 ** rng.uniform(-8, -1)
            chi = int(rng.integers(1, 40))
            k = mo.truncation_rank(s, chi, cut, mode)
            assert k == brute_rank(s, chi, cut, mode)
            assert mo.truncation_rank(s, chi, cut * 10, mode) <= k


# --------------------------------------------------- single-gate closed forms
def local(rng):
    return np.kron(cg.haar_unitary(rng, 2), cg.haar_unitary(rng, 2))


@pytest.mark.parametrize("abc", [(0.3, 0.2, 0.1), (0.7, 0.4, -0.2), (np.pi / 4, np.pi / 4, np.pi / 4),
                                 (np.pi / 4, 0.0, 0.0), (0.0, 0.0, 0.0)])
@pytest.mark.parametrize("side", ["out", "in"])
def test_single_gate_operator_schmidt_values(abc, side):
    rng = np.random.default_rng(5)
    g = local(rng) @ bf.kak_gate(*abc) @ local(rng)
    for n, bond in ((2, 0), (5, 2)):
        m = mo.OracleMPO(n)
        r = mo.bond_update(m, bond, g if side == "out" else None, g if side == "in" else None,
                           64, 1e-12, "rel_sv")
        want = bf.kak_schmidt_values(*abc)
        got = np.zeros(4)
        got[:len(r.s)] = r.s[:4]
        assert np.allclose(got, want, atol=1e-12)
        assert r.k == int(np.count_nonzero(want > 1e-12 * want[0]))


def test_swap_and_cnot_spectra():
    m = mo.OracleMPO(3)
    r = mo.bond_update(m, 1, mo.SWAP4, None, 64, 1e-12, "rel_sv")
    assert np.allclose(r.s, [0.5] * 4, atol=1e-14) and r.k == 4
    cnot = np.eye(4, dtype=complex)[[0, 1, 3, 2]]
    r = mo.bond_update(m, 0, None, cnot, 64, 1e-12, "rel_sv")
    assert r.k == 2 and np.allclose(r.s[:2], [np.sqrt(0.5)] * 2, atol=1e-14)


def test_mirrored_pair_on_identity_is_rank_one():
    rng = np.random.default_rng(2)
    g = cg.haar_su4(rng)
    m = mo.OracleMPO(4)
    r = mo.bond_update(m, 1, g.conj().T, g, 64, 1e-12, "rel_sv")
    assert r.k == 1 and abs(r.s[0] - 1) < 1e-13


# ------------------------------------------------- gate conventions vs dense
def random_mpo(n, seed, layers=3):
    rng = np.random.default_rng(seed)
    m = mo.OracleMPO(n)
    for l in range(layers):
        for i in range(l % 2, n - 1, 2):
            mo.commit(m, mo.bond_update(m, i, cg.haar_su4(rng), cg.haar_su4(rng), 256, 1e-14, "rel_sv"))
    return m


def embed(u, i, n):
    return np.kron(np.kron(np.eye(2 ** i), u), np.eye(2 ** (n - i - 2)))


@pytest.mark.parametrize("bond", [0, 2, 3])
def test_bond_update_equals_dense_products(bond):
    n = 5
    m = random_mpo(n, 10 + bond)
    before = m.dense_operator()
    rng = np.random.default_rng(bond)
    go, gi = cg.haar_su4(rng), cg.haar_su4(rng)
    r = mo.bond_update(m, bond, go, gi, 1024, 0.0, "weight")
    mo.commit(m, r)
    after = m.dense_operator()
    want = embed(go, bond, n) @ before @ embed(gi, bond, n)
    assert np.allclose(after, want, atol=1e-12)
    # the kept values are the operator-Schmidt values of the new operator at that cut
    vec = m.dense_vector().reshape(4 ** (bond + 1), -1)
    assert np.allclose(np.linalg.svd(vec, compute_uv=False)[:r.k], r.s[:r.k], atol=1e-12)
    # canonical form survives: every B is right-canonical
    for b in m.B:
        mat = b.reshape(b.shape[0], -1)
        assert np.allclose(mat @ mat.conj().T, np.eye(b.shape[0]), atol=1e-12)


def test_identity_mpo_is_identity_operator():
    m = mo.OracleMPO(4)
    assert np.allclose(m.dense_operator() * 2 ** 2, np.eye(16))
    assert m.size() == 16 and m.bond_dims() == [1, 1, 1]


# ----------------------------------------------- whole contraction (Alg. 1)
@pytest.mark.parametrize("reading", ["A", "B"])
def test_contraction_reproduces_dense_unitary(reading):
    c = cg.mirrored_peaked_circuit(8, 4, 21, reading=reading)
    res = mo.contract(c.n, c.gates, mo.OracleConfig(chi_max=256, cutoff=1e-12, unswap="none"))
    full = mo.full_operator(res) * 2 ** (c.n / 2)
    assert np.allclose(full, bf.circuit_unitary(c.n, c.gates), atol=1e-10)
    # unitarity bookkeeping: every update keeps sum s^2 = 1 when nothing is discarded
    for t in res.trace:
        if "k" in t:
            assert abs(t["total"] - 1.0) < 1e-10


def test_discarded_weight_bounds_the_error():
    c = cg.mirrored_peaked_circuit(8, 4, 22, reading="B")
    exact = bf.circuit_unitary(c.n, c.gates) / 2 ** (c.n / 2)
    res = mo.contract(c.n, c.gates, mo.OracleConfig(chi_max=6, cutoff=1e-12, unswap="none"))
    err = np.linalg.norm(mo.full_operator(res) - exact)
    bound = sum(np.sqrt(t["discarded"]) for t in res.trace if "k" in t)
    assert bound > 1e-3          # truncation really happened
    assert err <= bound * 1.01 + 1e-10


def test_collapse_invariant_of_the_unobfuscated_mirror():
    c = cg.mirror_only_circuit(10, 6, 3)
    res = mo.contract(c.n, c.gates, mo.OracleConfig(chi_max=64, cutoff=1e-12, unswap="none"))
    ups = [t for t in res.trace if "k" in t]
    assert len(ups) == len(c.gates) // 2
    assert all(t["k"] == 1 and abs(t["s"][0] - 1) < 1e-12 for t in ups)


@pytest.mark.parametrize("schedule", ["sequential", "parallel"])
@pytest.mark.parametrize("relaxed", [False, True])
def test_unswap_reconstructs_operator_and_rewiring_is_exact(schedule, relaxed):
    c = cg.mirrored_peaked_circuit(8, 3, 31, reading="B")
    cfg = mo.OracleConfig(chi_max=256, cutoff=1e-12, tau=300, unswap=schedule, relaxed=relaxed)
    ct = mo.Contraction(c.n, c.gates, cfg)
    checked = 0
    while ct.left or ct.right:
        ct.absorb_step()
        while ct.m.size() < cfg.tau and (ct.left or ct.right):
            ct.absorb_step()
        before = mo.full_operator(mo.OracleResult(None, 0, 0, None, list(ct.lay_l.site_of),
                                                  list(ct.lay_r.site_of), [], ct.m))
        dims0 = sum(ct.m.bond_dims())
        log = ct.unswap()
        after = mo.full_operator(mo.OracleResult(None, 0, 0, None, list(ct.lay_l.site_of),
                                                 list(ct.lay_r.site_of), [], ct.m))
        assert np.allclose(before, after, atol=1e-10)           # M = P_L M~ P_R
        if not relaxed:
            assert sum(ct.m.bond_dims()) <= dims0
        checked += len(log)
    assert checked > 0
    site_bits, p, n2 = mo.extract_peak(ct.m)
    res = mo.OracleResult(None, p, n2, site_bits, list(ct.lay_l.site_of), list(ct.lay_r.site_of), [], ct.m)
    full = mo.full_operator(res) * 2 ** (c.n / 2)
    assert np.allclose(full, bf.circuit_unitary(c.n, c.gates), atol=1e-9)


@pytest.mark.parametrize("side,freq", [("adaptive", (1, 1)), ("fixed", (2, 1)), ("fixed", (1, 3))])
def test_side_selection_reproduces_dense_unitary(side, freq):
    """App. A.3: whichever side each step takes, and with unswapping and
    rewiring between the phases, the contracted operator P_L M~ P_R is the
    circuit's unitary (no truncation); every gate is absorbed exactly once."""
    c = cg.mirrored_peaked_circuit(8, 3, 41, reading="B")
    cfg = mo.OracleConfig(chi_max=256, cutoff=1e-12, tau=300, unswap="parallel", side=side, fixed_freq=freq)
    ct = mo.Contraction(c.n, c.gates, cfg)
    res = ct.run()
    full = mo.full_operator(res) * 2 ** (c.n / 2)
    assert np.allclose(full, bf.circuit_unitary(c.n, c.gates), atol=1e-9)
    absorbed = sum(1 for t in res.trace if t.get("stage") == "absorb")
    fused = sum(1 for t in res.trace if t.get("stage") == "absorb" and t.get("fused"))
    assert absorbed + fused == len(c.gates)
    if side == "fixed":
        # while both sides have layers, the period is f_L steps of C_L then f_R of C_R
        sides = [t["taken"] for t in res.trace if t.get("stage") == "layer"]
        fl, fr = freq
        nl = nr = len(mo.asap_layers(c.gates, c.n)) // 2
        left = right = 0
        for j, x in enumerate(sides):
            if left >= nl or right >= nr:
                break
            assert x == ("L" if j % (fl + fr) < fl else "R")
            left += x == "L"
            right += x == "R"
        assert j >= fl + fr


def test_adaptive_keeps_the_smaller_copy_and_changes_the_path():
    """App. A.3: each adaptive step keeps the copy with the smaller size(M)
    (ties: the left one), and the kept size is the MPO's size after the step;
    on this circuit the adaptive path differs from Alg. 1's alternation but
    ends at the same operator."""
    c = cg.mirrored_peaked_circuit(8, 3, 43, reading="B")
    base = dict(chi_max=256, cutoff=1e-12, tau=400, unswap="parallel")
    ct = mo.Contraction(c.n, c.gates, mo.OracleConfig(side="adaptive", **base))
    res = ct.run()
    picks = [t for t in res.trace if t.get("stage") == "side"]
    assert picks and any(t["side"] == "R" for t in picks) and any(t["side"] == "L" for t in picks)
    for j, t in enumerate(res.trace):
        if t.get("stage") != "side":
            continue
        kept = min(t["size_left"], t["size_right"])
        assert t["side"] == ("L" if t["size_left"] <= t["size_right"] else "R")
        prev = [u for u in res.trace[:j] if "size" in u and u.get("stage") != "unswap"]
        assert prev and prev[-1]["size"] == kept
    alt = mo.contract(c.n, c.gates, mo.OracleConfig(side="both", **base))
    assert np.allclose(mo.full_operator(res), mo.full_operator(alt), atol=1e-10)


def test_unswap_removes_a_bare_swap_layer():
    n = 7
    m = mo.OracleMPO(n)
    for i in range(0, n - 1, 2):
        mo.commit(m, mo.bond_update(m, i, mo.SWAP4, None, 64, 1e-12, "rel_sv"))
    for i in range(1, n - 1, 2):
        mo.commit(m, mo.bond_update(m, i, None, mo.SWAP4, 64, 1e-12, "rel_sv"))
    assert max(m.bond_dims()) == 4
    for sched in ("sequential", "parallel"):
        mm = m.copy()
        cfg = mo.OracleConfig(chi_max=64, cutoff=1e-12, unswap=sched)
        log = (mo.unswap_sequential if sched == "sequential" else mo.unswap_parallel)(mm, cfg)
        assert mm.bond_dims() == [1] * (n - 1) and len(log) == n - 1


# ------------------------------------------------------- peak extraction
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_extraction_matches_statevector_brute_force(seed):
    c = cg.mirrored_peaked_circuit(9, 3, 40 + seed)
    res = mo.contract(c.n, c.gates, mo.OracleConfig(chi_max=256, cutoff=1e-12, tau=400, unswap="parallel"))
    psi = bf.circuit_state(c.n, c.gates)
    prob = np.abs(psi) ** 2
    best = int(np.argmax(prob))
    assert (res.bits == bf.bits_of(best, c.n)).all()
    assert (res.bits == c.peak).all()
    assert abs(res.prob - prob[best]) < 1e-10
    assert abs(res.norm2 - 2.0 ** -c.n) < 1e-12 * 2.0 ** -c.n * 100


@pytest.mark.parametrize("seed", [3, 8])
def test_sampling_is_inverse_cdf_of_the_statevector(seed):
    """Sec. II.C sampling, pinned by brute force: with the same uniforms, the
    oracle's sampled strings equal those of sequential inverse-CDF sampling
    from the dense state's marginals (bit i = 0 iff u_i < P(x_i = 0 | x_<i)),
    and each returned probability is |<x|psi>|^2 / <psi|psi>."""
    c = cg.mirrored_peaked_circuit(8, 3, 60 + seed, reading="B")
    res = mo.contract(c.n, c.gates, mo.OracleConfig(chi_max=256, cutoff=1e-12, tau=300, unswap="parallel"))
    psi = bf.circuit_state(c.n, c.gates)
    # the MPS's site i carries the output leg of logical qubit logical_at[i]
    logical_at = np.argsort(res.layout_left)
    assert not np.array_equal(logical_at, np.arange(c.n))        # unswapping moved qubits
    pr = (np.abs(psi) ** 2).reshape([2] * c.n).transpose(logical_at).reshape(-1)   # axes in site order
    pr = pr / pr.sum()
    rng = np.random.default_rng(seed)
    u = rng.random((200, c.n))
    bits, probs = mo.sample(res.mpo, u)
    for s in range(u.shape[0]):
        prefix = ()
        for i in range(c.n):
            marg = pr.reshape([2] * c.n)[prefix].reshape(2, -1).sum(axis=1)
            x = 0 if u[s, i] < marg[0] / marg.sum() else 1
            assert bits[s, i] == x
            prefix = prefix + (x,)
        idx = int("".join(map(str, bits[s])), 2)
        assert abs(probs[s] - pr[idx]) <= 1e-10
    # the peak is the most frequent string for a peaked state
    assert len({tuple(b) for b in bits}) > 1


def test_extraction_probability_of_returned_string_is_exact():
    # on a generic (not peaked) MPO the greedy string need not be the argmax,
    # but the returned probability must be that string's exact weight
    rng = np.random.default_rng(3)
    n = 6
    m = random_mpo(n, 77, layers=4)
    bits, p, n2 = mo.extract_peak(m)
    op = m.dense_operator()
    psi = op[:, 0]
    idx = int("".join(str(int(b)) for b in bits), 2)
    assert abs(p - abs(psi[idx]) ** 2 / np.vdot(psi, psi).real) < 1e-12
    assert abs(n2 - np.vdot(psi, psi).real) < 1e-14


@pytest.mark.parametrize("n", [2, 3, 4, 5, 8, 9])
def test_closed_form_peak_probability_vs_statevector(n):
    c = cg.mirrored_peaked_circuit(n, 2, 11 + n)
    psi = bf.circuit_state(n, c.k_gates)
    assert abs(bf.peak_probability_closed_form(n, c.k_gates) - abs(psi[0]) ** 2) < 1e-13
    full = bf.circuit_state(n, c.gates)
    idx = int(c.peak_string, 2)
    assert abs(abs(full[idx]) ** 2 - abs(psi[0]) ** 2) < 1e-12


@pytest.mark.parametrize("n", [4, 7, 10])
def test_k_margins_vs_statevector(n):
    c = cg.mirrored_peaked_circuit(n, 2, 60 + n)
    psi = np.abs(bf.circuit_state(n, c.k_gates).reshape([2] * n)) ** 2
    got = bf.k_state_margins(n, c.k_gates)
    for i in range(n):
        pre = psi[(0,) * i]
        marg = pre.reshape(2, -1).sum(axis=1)
        assert abs(got[i] - marg[0] / marg.sum()) < 1e-12


@pytest.mark.parametrize("config", [0, 1, 2])
def test_workload_peaks_are_greedy_readable(config):
    c = cg.config_circuit(config)
    assert bf.k_state_margins(c.n, c.k_gates).min() > 0.5
    p = bf.peak_probability_closed_form(c.n, c.k_gates)
    assert 1e-5 < p < 1


def test_batching_workload_peaks_are_greedy_readable():
    """All 128 circuits of the batching workload: every prefix conditional of
    K|0> along 0...0 exceeds 1/2 (the oracle's own computation), so the greedy
    readout lands on the planted b."""
    work = cg.batch_workload()
    assert len(work) == 128
    for c, chi in work:
        assert chi in (128, 256, 512)
        assert bf.k_state_margins(c.n, c.k_gates).min() > 0.5


@pytest.mark.parametrize("rate", [1, 4, 16])
def test_serving_workload_peaks_are_greedy_readable(rate):
    """The first arrivals of each serving rate (n in {24, 40, 56})."""
    from paper_2604_21908_amd import serve
    reqs = serve.poisson_requests(rate, 600)[:12]
    serve.prepare(reqs)
    for r in reqs:
        assert r.circuit.n == r.n and r.n in (24, 40, 56)
        assert bf.k_state_margins(r.n, r.circuit.k_gates).min() > 0.5


@pytest.mark.parametrize("n", [2, 3, 6, 9, 12])
def test_generator_admission_check_matches_oracle(n):
    """The generator's own prefix conditionals of K|0> (an exact chain rewrite)
    equal the oracle's (truncation-free splits and environments) and, for
    n <= 12, the statevector's."""
    c = cg.mirrored_peaked_circuit(n, 2, 90 + n, min_margin=0.0)
    layers = [[g for g in c.k_gates if g[0] % 2 == 0], [g for g in c.k_gates if g[0] % 2 == 1]]
    got = cg.k_prefix_conditionals(n, layers)
    assert np.max(np.abs(got - bf.k_state_margins(n, c.k_gates))) < 1e-12
    psi = np.abs(bf.circuit_state(n, c.k_gates).reshape([2] * n)) ** 2
    for i in range(n):
        marg = psi[(0,) * i].reshape(2, -1).sum(axis=1)
        assert abs(got[i] - marg[0] / marg.sum()) < 1e-12


def test_generator_redraws_k_below_the_margin():
    """A margin no K can meet makes the generator give up loudly; a seed whose
    first K fails the 1/2 margin gets a different, admissible K."""
    with pytest.raises(RuntimeError):
        cg.mirrored_peaked_circuit(6, 2, 5, min_margin=1.0, max_k_draws=3)
    n, kw = 24, dict(with_swaps=False, dress=False)
    first_fail = None
    for seed in range(40):
        c0 = cg.mirrored_peaked_circuit(n, 1, seed, min_margin=0.0, **kw)
        if bf.k_state_margins(n, c0.k_gates).min() <= 0.5:
            first_fail = seed
            break
    assert first_fail is not None
    c = cg.mirrored_peaked_circuit(n, 1, first_fail, **kw)
    assert bf.k_state_margins(n, c.k_gates).min() > 0.5
    assert c.digest() != c0.digest()


# ------------------------------------------------ planted mistakes must fail
def test_planted_mistakes_are_caught(monkeypatch):
    """A transposed input gate, a dropped Lambda or a dropped conjugate in the
    oracle each break the dense pin above."""
    n, bond = 5, 2
    m = random_mpo(n, 12)
    before = m.dense_operator()
    rng = np.random.default_rng(0)
    go, gi = cg.haar_su4(rng), cg.haar_su4(rng)
    want = embed(go, bond, n) @ before @ embed(gi, bond, n)

    def run():
        mm = m.copy()
        mo.commit(mm, mo.bond_update(mm, bond, go, gi, 1024, 0.0, "weight"))
        return np.allclose(mm.dense_operator(), want, atol=1e-10)

    assert run()
    orig = mo.apply_gates_to_theta
    monkeypatch.setattr(mo, "apply_gates_to_theta", lambda t, a, b: orig(t, a, None if b is None else b.T))
    assert not run()
    monkeypatch.setattr(mo, "apply_gates_to_theta", lambda t, a, b: orig(t, a, None if b is None else b.conj()))
    assert not run()
    monkeypatch.setattr(mo, "apply_gates_to_theta", lambda t, a, b: orig(t, b, a))
    assert not run()


# ---------------------------------------------- all-to-all input, eager rewiring
@pytest.mark.parametrize("reading", ["A", "B"])
def test_all_to_all_generator_is_planted(reading):
    """Gates on arbitrary pairs (random matchings, selection-sort SWAPs):
    the circuit operator is still X^b K, so the statevector's argmax is b
    with the closed-form probability."""
    c = cg.mirrored_peaked_circuit(8, 3, 5, reading=reading, connectivity="all")
    assert sum(1 for q0, q1, _ in c.gates if abs(q0 - q1) > 1) > 5
    psi = bf.circuit_state(c.n, c.gates)
    idx = int(np.argmax(np.abs(psi) ** 2))
    assert np.array_equal(bf.bits_of(idx, c.n), c.peak)
    assert abs(abs(psi[idx]) ** 2 - bf.peak_probability_closed_form(c.n, c.k_gates)) < 1e-12


@pytest.mark.parametrize("router", ["up", "middle"])
def test_transpile_linear_is_nearest_neighbour_and_exact(router):
    """Alg. 1 step 1: the transpiled half is nearest-neighbour on the sites,
    and replaying it on a dense state (circuit gates on their logical qubits,
    SWAPs exchanging the two logical qubits' sites) equals the original
    gates followed by the permutation the SWAPs made."""
    rng = np.random.default_rng(4)
    n = 6
    gates = [(int(a), int(b), cg.haar_su4(rng), j)
             for j, (a, b) in enumerate(rng.permuted(np.tile(np.arange(n), (8, 1)), axis=1)[:, :2])]
    lay = mo.Layout(n)
    layers = mo.transpile_linear(gates, lay, router)
    site_of, logical_at = list(range(n)), list(range(n))
    seen = []
    for layer in layers:
        used = set()
        for (a, b, u, is_swap, gid) in layer:
            sa, sb = site_of[a], site_of[b]
            assert abs(sa - sb) == 1 and not ({sa, sb} & used)
            used |= {sa, sb}
            if is_swap:
                logical_at[sa], logical_at[sb] = b, a
                site_of[a], site_of[b] = sb, sa
            else:
                seen.append(gid)
    assert sorted(seen) == list(range(len(gates)))       # every gate once (ASAP may reorder commuting ones)
    # dense check: apply the entries in layer order on site-indexed qubits
    psi = bf.circuit_state(n, [])
    site_of = list(range(n))
    for layer in layers:
        for (a, b, u, is_swap, gid) in layer:
            sa, sb = site_of[a], site_of[b]
            if is_swap:
                psi = bf.apply_gate_state(psi.reshape([2] * n), n, sa, sb, mo.SWAP4).reshape(-1)
                site_of[a], site_of[b] = sb, sa
            else:
                psi = bf.apply_gate_state(psi.reshape([2] * n), n, sa, sb, u).reshape(-1)
    ref = bf.circuit_state(n, [(a, b, u) for (a, b, u, _) in gates])
    # ref is on logical qubits; psi on sites: logical q sits at site site_of[q]
    ref_sites = ref.reshape([2] * n).transpose(np.argsort(site_of)).reshape(-1)
    assert np.allclose(psi, ref_sites, atol=1e-12)


@pytest.mark.parametrize("router", ["up", "middle"])
@pytest.mark.parametrize("side", ["both", "adaptive"])
@pytest.mark.parametrize("reading", ["A", "B"])
def test_eager_rewiring_reproduces_dense_unitary(side, reading, router):
    """Alg. 1 with eager rewiring (transpile, strip the transpilation SWAPs
    after unswapping, reindex, re-transpile) on an all-to-all circuit: the
    contracted operator is the circuit's unitary, the peak is b."""
    c = cg.mirrored_peaked_circuit(6, 2, 5, reading=reading, connectivity="all")
    for rewire in ("lazy", "eager"):
        res = mo.contract(c.n, c.gates, mo.OracleConfig(chi_max=256, cutoff=1e-12, tau=200, unswap="parallel",
                                                        rewire=rewire, side=side, router=router))
        full = mo.full_operator(res) * 2 ** (c.n / 2)
        assert np.allclose(full, bf.circuit_unitary(c.n, c.gates), atol=1e-9), rewire
        assert np.array_equal(res.bits, c.peak)
        assert any(t.get("stage") == "unswap" and t["accepted"] for t in res.trace)
