"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here re-types the oracle's formulas: the expected values come from the
paper's printed examples (``tests/golden/``), from closed forms, from a
set-based brute force that never uses the digit arithmetic of rho, and from
invariants of the prime-implicant set.
"""
import itertools
import math
import os
import random

import numpy as np
import pytest

import oracle
from paper_2302_10083_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def both_oracles(n, tt):
    """(M, O) as sets from the definitional enumerator and from brute force;
    asserts they agree."""
    M2, O2, _ = oracle.primes(n, tt)
    M1, O1 = oracle.bruteforce(n, tt)
    assert np.array_equal(M1, M2), "brute force and enumerator disagree on M"
    assert np.array_equal(O1, O2), "brute force and enumerator disagree on O"
    return oracle.bitmap_to_set(n, M2), oracle.bitmap_to_set(n, O2)


def strings(n, rhos):
    return sorted(oracle.string_of(n, r) for r in rhos)


# ----------------------------------------------------------------------------
# paper's printed examples


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_majority_example():
    rows = _read_golden("maj3.txt")
    n = int(rows[0][1])
    expected = sorted(r[1] for r in rows if r[0] == "prime")
    tt = inputs.interval(n, 2, n)  # majority of 3: at least two ones
    M, O = both_oracles(n, tt)
    assert strings(n, O) == expected
    # the minterms of Maj plus the three primes are all the implicants
    minterms = {"110", "101", "011", "111"}
    assert set(strings(n, M)) == minterms | set(expected)


def test_string_examples():
    rows = _read_golden("string_examples.txt")
    # x_1 x_3' for n = 5
    n = int(rows[0][1])
    prod = rows[1][1]
    care = sum(1 << i for i, c in enumerate(prod) if c != "*")
    val = sum(1 << i for i, c in enumerate(prod) if c == "1")
    assert care == 0b00101 and val == 0b00001  # literals on x_1 (positive), x_3 (negated)
    tt = inputs.from_terms(n, [(care, val)])
    _, O = both_oracles(n, tt)
    assert strings(n, O) == [prod]
    # 0011* + 0111* = 0*11*
    n = int(rows[2][1])
    a, b = rows[3][1], rows[3][2]
    merged = rows[4][1]
    terms = []
    for s in (a, b):
        terms.append((sum(1 << i for i, c in enumerate(s) if c != "*"),
                      sum(1 << i for i, c in enumerate(s) if c == "1")))
    tt = inputs.from_terms(n, terms)
    M, O = both_oracles(n, tt)
    assert strings(n, O) == [merged]
    assert oracle.rho_of(a) in M and oracle.rho_of(b) in M


@pytest.mark.parametrize("n", list(range(0, 9)))
def test_constant_one_only_allstar_prime(n):
    rows = _read_golden("constant_one.txt")
    assert rows[1][1] == "all-star"
    M, O = both_oracles(n, inputs.constant(n, 1))
    assert M == set(range(3**n))
    assert O == {3**n - 1}
    assert strings(n, O) == ["*" * n]


@pytest.mark.parametrize("n", [10, 12])
def test_constant_one_enum_larger(n):
    M, O, lst = oracle.primes(n, inputs.constant(n, 1))
    assert int(np.bitwise_count(M).sum()) == 3**n
    assert lst.tolist() == [3**n - 1]


@pytest.mark.parametrize("n", list(range(0, 9)))
def test_constant_zero_no_primes(n):
    M, O = both_oracles(n, inputs.constant(n, 0))
    assert M == set() and O == set()


# ----------------------------------------------------------------------------
# set-based brute force: cubes as sets of minterms, no rho digit arithmetic


def _cube_minterm_sets(n):
    """For every string s in {0,1,*}^n (s_1 first), the frozenset of the x it
    covers, where x_i = bit i-1 of x."""
    out = {}
    for s in itertools.product("01*", repeat=n):
        choices = [(0,) if c == "0" else (1,) if c == "1" else (0, 1) for c in s]
        xs = frozenset(sum(b << i for i, b in enumerate(bits)) for bits in itertools.product(*choices))
        out["".join(s)] = xs
    return out


def _setwise_primes(n, support, cubes):
    impl = {s for s, xs in cubes.items() if xs <= support}
    primes = {s for s in impl if not any(cubes[s] < cubes[t] for t in impl)}
    return impl, primes


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_all_functions_small_n_vs_setwise(n):
    cubes = _cube_minterm_sets(n)
    for f in range(1 << (1 << n)):
        support = frozenset(x for x in range(1 << n) if (f >> x) & 1)
        bits = np.array([(f >> x) & 1 for x in range(1 << n)], dtype=bool)
        tt = inputs.from_bits(n, bits)
        impl, primes = _setwise_primes(n, support, cubes)
        M, O = both_oracles(n, tt)
        assert strings(n, M) == sorted(impl), f
        assert strings(n, O) == sorted(primes), f


def test_random_functions_n4_n5_vs_setwise():
    rng = random.Random(4)
    for n, count in ((4, 120), (5, 25)):
        cubes = _cube_minterm_sets(n)
        for _ in range(count):
            bits = np.array([rng.random() < rng.choice([0.3, 0.6, 0.85]) for _ in range(1 << n)])
            support = frozenset(int(x) for x in np.nonzero(bits)[0])
            tt = inputs.from_bits(n, bits)
            impl, primes = _setwise_primes(n, support, cubes)
            M, O = both_oracles(n, tt)
            assert strings(n, M) == sorted(impl)
            assert strings(n, O) == sorted(primes)


# ----------------------------------------------------------------------------
# closed forms


@pytest.mark.parametrize("n", list(range(1, 11)))
def test_parity_primes_are_odd_minterms(n):
    # no two true minterms of parity are adjacent, so no merge ever happens
    M2, O2, lst = oracle.primes(n, inputs.parity(n))
    odd = sorted(sum(((x >> i) & 1) * 3**i for i in range(n)) for x in range(1 << n) if bin(x).count("1") % 2)
    assert lst.tolist() == odd
    assert np.array_equal(M2, O2)
    if n <= 8:
        M1, O1 = oracle.bruteforce(n, inputs.parity(n))
        assert np.array_equal(O1, O2)


def _interval_expected(n, a, b):
    """Symmetric f = [a <= |x| <= b].  A cube with o ones and k stars covers
    weights o..o+k: it is an implicant iff a <= o and o + k <= b, and prime iff
    moreover no literal can be dropped, i.e. o = a and o + k = b."""
    M, O = set(), set()
    for s in itertools.product("01*", repeat=n):
        o, k = s.count("1"), s.count("*")
        r = oracle.rho_of("".join(s))
        if a <= o and o + k <= b:
            M.add(r)
            if o == a and o + k == b:
                O.add(r)
    return M, O


@pytest.mark.parametrize("n,a,b", [(3, 2, 3), (4, 1, 2), (5, 0, 3), (5, 2, 2), (6, 1, 4), (6, 3, 6), (7, 2, 5), (8, 0, 8)])
def test_interval_symmetric_closed_form(n, a, b):
    M_exp, O_exp = _interval_expected(n, a, b)
    M, O = both_oracles(n, inputs.interval(n, a, b))
    assert M == M_exp
    assert O == O_exp
    assert len(O) == math.comb(n, a) * math.comb(n - a, b - a)


@pytest.mark.parametrize("n,a,b", [(12, 4, 9), (13, 6, 7), (14, 2, 12)])
def test_interval_symmetric_counts_larger(n, a, b):
    _, O, lst = oracle.primes(n, inputs.interval(n, a, b))
    assert len(lst) == math.comb(n, a) * math.comb(n - a, b - a)
    for r in lst[:: max(1, len(lst) // 200)]:
        s = oracle.string_of(n, int(r))
        assert s.count("1") == a and s.count("*") == b - a


@pytest.mark.parametrize("seed", range(6))
def test_single_product_term(seed):
    rng = random.Random(seed)
    n = rng.randint(1, 9)
    care = rng.getrandbits(n)
    val = rng.getrandbits(n) & care
    tt = inputs.from_terms(n, [(care, val)])
    M, O = both_oracles(n, tt)
    term = "".join(("1" if (val >> i) & 1 else "0") if (care >> i) & 1 else "*" for i in range(n))
    assert strings(n, O) == [term]
    # implicants: agree with the term on its literals, anything elsewhere
    assert len(M) == 3 ** (n - bin(care).count("1"))


def _unate_expected(n, terms):
    """Prime implicants of a unate DNF: the terms left after absorption (a term
    whose literal set contains another term's literal set is dropped)."""
    ts = sorted(set(terms))
    keep = [t for t in ts if not any(u != t and (u[0] & t[0]) == u[0] for u in ts)]
    out = set()
    for care, val in keep:
        s = "".join(("1" if (val >> i) & 1 else "0") if (care >> i) & 1 else "*" for i in range(n))
        out.add(oracle.rho_of(s))
    return out


@pytest.mark.parametrize("n,T,wlo,whi,seed", [(6, 5, 1, 4, 1), (8, 12, 2, 5, 2), (10, 30, 2, 6, 3), (12, 60, 3, 8, 4), (14, 80, 4, 9, 5)])
def test_unate_dnf_primes_are_absorbed_terms(n, T, wlo, whi, seed):
    terms = inputs.unate_terms(n, T, wlo, whi, seed)
    tt = inputs.from_terms(n, terms)
    _, O, lst = oracle.primes(n, tt)
    assert set(int(x) for x in lst) == _unate_expected(n, terms)
    if n <= 8:
        M1, O1 = oracle.bruteforce(n, tt)
        assert np.array_equal(O1, O)


# ----------------------------------------------------------------------------
# invariants and cross-checks on random functions


def _covers(n, big, small):
    """True iff cube `big` contains cube `small` (string-wise)."""
    sb, ss = oracle.string_of(n, big), oracle.string_of(n, small)
    return all(a == "*" or a == b for a, b in zip(sb, ss))


@pytest.mark.parametrize("n,p,seed", [(6, 0.5, 1), (7, 0.8, 2), (8, 0.9, 3), (8, 0.3, 4)])
def test_invariants_random(n, p, seed):
    tt = inputs.bernoulli(n, p, seed)
    M, O = both_oracles(n, tt)
    bits = inputs.to_bits(n, tt)
    # M restricted to minterms is the truth table
    binary = {sum(((x >> i) & 1) * 3**i for i in range(n)) for x in range(1 << n)}
    assert {r for r in M if r in binary} == {sum(((x >> i) & 1) * 3**i for i in range(n)) for x in range(1 << n) if bits[x]}
    assert O <= M
    # antichain: no prime strictly contains another
    Ol = sorted(O)
    for a in Ol:
        for b in Ol:
            if a != b:
                assert not _covers(n, a, b)
    # down-closure of the primes is exactly the implicant set
    for r in M:
        assert any(_covers(n, p_, r) for p_ in Ol)
    # every true minterm is covered by a prime (covering invariant)
    for x in np.nonzero(bits)[0]:
        r = sum(((int(x) >> i) & 1) * 3**i for i in range(n))
        assert any(_covers(n, p_, r) for p_ in Ol)


@pytest.mark.parametrize("n,p,seed", [(9, 0.5, 11), (10, 0.9, 12), (11, 0.7, 13), (12, 0.95, 14), (12, 0.5, 15)])
def test_bruteforce_vs_enumerator_random(n, p, seed):
    tt = inputs.bernoulli(n, p, seed)
    both_oracles(n, tt)


@pytest.mark.parametrize("n,seed", [(4, 21), (5, 22), (6, 23)])
def test_one_step_prime_equals_all_divisor_prime(n, seed):
    tt = inputs.bernoulli(n, 0.75, seed)
    _, O1 = oracle.bruteforce(n, tt, all_divisors=False)
    _, Oa = oracle.bruteforce(n, tt, all_divisors=True)
    assert np.array_equal(O1, Oa)


def _permute_tt(n, tt, perm):
    """g(x) = f(y) where y_{perm[i]} = x_i."""
    bits = inputs.to_bits(n, tt)
    out = np.zeros(1 << n, dtype=bool)
    for x in range(1 << n):
        y = 0
        for i in range(n):
            if (x >> i) & 1:
                y |= 1 << perm[i]
        out[x] = bits[y]
    return inputs.from_bits(n, out)


@pytest.mark.parametrize("n,seed", [(6, 31), (8, 32), (9, 33)])
def test_equivariance_permutation_and_negation(n, seed):
    rng = random.Random(seed)
    tt = inputs.bernoulli(n, 0.8, seed)
    _, _, lst = oracle.primes(n, tt)
    base = set(strings(n, [int(r) for r in lst]))
    perm = list(range(n))
    rng.shuffle(perm)
    _, _, lst_p = oracle.primes(n, _permute_tt(n, tt, perm))
    # digit i of a prime of g is digit perm[i] of a prime of f
    mapped = {"".join(s[perm[i]] for i in range(n)) for s in base}
    assert set(strings(n, [int(r) for r in lst_p])) == mapped
    # negating x_j swaps digits 0 and 1 at position j
    j = rng.randrange(n)
    bits = inputs.to_bits(n, tt)
    neg = inputs.from_bits(n, bits[np.arange(1 << n) ^ (1 << j)])
    _, _, lst_n = oracle.primes(n, neg)
    sw = {"0": "1", "1": "0", "*": "*"}
    mapped_n = {s[:j] + sw[s[j]] + s[j + 1:] for s in base}
    assert set(strings(n, [int(r) for r in lst_n])) == mapped_n


def test_extract_ascending_and_capped():
    n = 7
    tt = inputs.bernoulli(n, 0.85, 7)
    _, O, lst = oracle.primes(n, tt)
    assert np.all(np.diff(lst.astype(np.int64)) > 0)
    part, cnt = oracle.extract(n, O, cap=5)
    assert cnt == len(lst) and part.tolist() == lst[:5].tolist()


def test_per_cube_definitions_match_bitmaps():
    n = 9
    tt = inputs.dnf(n, 12, 2, 5, 99)
    M, O, _ = oracle.primes(n, tt)
    Ms, Os = oracle.bitmap_to_set(n, M), oracle.bitmap_to_set(n, O)
    rng = random.Random(5)
    for _ in range(400):
        r = rng.randrange(3**n)
        assert oracle.is_implicant(n, tt, r) == (r in Ms)
        assert oracle.is_prime(n, tt, r) == (r in Os)


def test_sample_matches_bitmaps():
    n = 10
    tt = inputs.bernoulli(n, 0.88, 1234)
    M, O, _ = oracle.primes(n, tt)
    rng = np.random.default_rng(3)
    rhos = rng.integers(0, 3**n, size=3000, dtype=np.uint64)
    pr, _ = oracle.sample(n, tt, rhos, "prime")
    im, _ = oracle.sample(n, tt, rhos, "implicant")
    Os, Ms = oracle.bitmap_to_set(n, O), oracle.bitmap_to_set(n, M)
    assert [bool(int(r) in Os) for r in rhos] == pr.tolist()
    assert [bool(int(r) in Ms) for r in rhos] == im.tolist()


# --- complement mode (Sec. 1, "New method": primes of NOT f give f's CNF) ---

def _complement(n, tt):
    c = ~np.asarray(tt, dtype=np.uint32)
    if n < 5:
        c &= np.uint32((1 << (1 << n)) - 1)
    return c


def test_cnf_of_and2_golden():
    """f = x1 AND x2: NOT f = NOT x1 OR NOT x2 has the primes 0* and *0, the
    clauses x1 and x2 of f's CNF."""
    tt = np.array([0b1000], dtype=np.uint32)  # f(x) = 1 only at x = 3
    _, _, lst = oracle.primes(2, _complement(2, tt))
    assert [oracle.string_of(2, int(r)) for r in lst] == ["*0", "0*"]
    assert list(lst) == [oracle.rho_of("*0"), oracle.rho_of("0*")] == [2, 6]


@pytest.mark.parametrize("n,p,seed", [(3, 0.7, 1), (5, 0.8, 2), (7, 0.9, 3), (8, 0.95, 4), (9, 0.3, 5)])
def test_cnf_clauses_reproduce_f(n, p, seed):
    """Every prime s of NOT f gives the clause 'x is not covered by s'; f is
    the AND of these clauses (they are implied by f, and the primes of NOT f
    cover every zero of f)."""
    tt = inputs.bernoulli(n, p, seed)
    _, _, lst = oracle.primes(n, _complement(n, tt))
    f = np.array([(int(tt[x >> 5]) >> (x & 31)) & 1 for x in range(1 << n)], dtype=bool)
    conj = np.ones(1 << n, dtype=bool)
    for r in lst:
        s = oracle.string_of(n, int(r))
        covered = np.ones(1 << n, dtype=bool)
        xs = np.arange(1 << n)
        for i, ch in enumerate(s):
            if ch != "*":
                covered &= ((xs >> i) & 1) == int(ch)
        assert not np.any(covered & f), "a clause of f is violated by a true point"
        conj &= ~covered
    assert np.array_equal(conj, f)


def _restrict(n, t, tt, a_digits):
    """Truth table (bool array over x_1..x_m) of f_a: the AND of f over the
    minterms of the cube a on the top t variables."""
    m = n - t
    bits = np.unpackbits(np.asarray(tt, dtype=np.uint32).view(np.uint8), bitorder="little")[: 1 << n].astype(bool)
    out = np.ones(1 << m, dtype=bool)
    for xt in range(1 << t):
        if all(d == 2 or ((xt >> j) & 1) == d for j, d in enumerate(a_digits)):
            out &= bits[xt << m: (xt + 1) << m]
    return inputs.from_bits(m, out)


@pytest.mark.parametrize("n,t,p,seed", [(5, 1, 0.7, 1), (6, 2, 0.8, 2), (7, 3, 0.9, 3), (8, 2, 0.6, 4),
                                        (8, 4, 0.95, 5), (9, 1, 0.85, 6)])
def test_top_digit_slicing_identity(n, t, p, seed):
    """The decomposition the sliced GPU path relies on, checked with whole
    bitmaps: cube s.a (a on the top t variables) is prime for f exactly when
    s is prime for f_a and, for every binary digit j of a, s is not an
    implicant of f_{a[j <- *]}."""
    tt = inputs.bernoulli(n, p, 9100 + seed)
    _, O, _ = oracle.primes(n, tt)
    full = oracle.bitmap_to_set(n, O)
    m = n - t
    got = set()
    for idx in range(3**t):
        a = [(idx // 3**j) % 3 for j in range(t)]
        _, Oa, _ = oracle.primes(m, _restrict(n, t, tt, a))
        keep = oracle.bitmap_to_set(m, Oa)
        for j, d in enumerate(a):
            if d != 2:
                starred = list(a)
                starred[j] = 2
                Mj = oracle.enum_M(m, _restrict(n, t, tt, starred))
                keep -= oracle.bitmap_to_set(m, Mj)
        got |= {s + idx * 3**m for s in keep}
    assert got == full
    assert len(full) > 0


@pytest.mark.parametrize("n,kind,seed", [(5, 0.7, 1), (6, 0.85, 2), (7, "dnf", 3), (8, 0.95, 4)])
def test_sibling_form_of_the_reduce(n, kind, seed):
    """The derived identity the merge+reduce column pass uses: for a cube s
    with digit i binary and s' the cube with that digit flipped,
    M(s[i <- *]) = M(s) AND M(s') (the Lemma of Sec. 4.1), so reducing with
    the sibling's M gives the same O as reducing with the star neighbour's."""
    if kind == "dnf":
        tt = inputs.dnf(n, 6, 1, 4, 9300 + seed)
    else:
        tt = inputs.bernoulli(n, kind, 9300 + seed)
    M = np.zeros(3**n, dtype=bool)
    M[sorted(oracle.bitmap_to_set(n, oracle.enum_M(n, tt)))] = True
    rho = np.arange(3**n, dtype=np.int64)
    p3 = 3 ** np.arange(n, dtype=np.int64)
    digs = (rho[:, None] // p3[None, :]) % 3
    by_star, by_sib = M.copy(), M.copy()
    for i in range(n):
        s = rho[digs[:, i] != 2]
        d = digs[s, i]
        star = s + (2 - d) * p3[i]
        sib = s + (1 - 2 * d) * p3[i]
        assert np.array_equal(M[star], M[s] & M[sib])
        by_star[s] &= ~M[star]
        by_sib[s] &= ~M[sib]
    _, O, _ = oracle.primes(n, tt)
    assert np.array_equal(by_star, by_sib)
    assert set(np.flatnonzero(by_sib).tolist()) == oracle.bitmap_to_set(n, O)
    assert by_sib.any() and (M & ~by_sib).any()


@pytest.mark.parametrize("n,kind,seed", [(6, 0.8, 1), (7, "dnf", 2), (8, 0.9, 3), (9, "dnf", 4)])
def test_reduce_in_staged_one_step_groups(n, kind, seed):
    """Reading 7 as the final tile reduce uses it: the dimensions split into
    groups taken one after another, each group reduced in one step from the
    values the previous groups left (x loses its bit when S(x[i <- *]) is set
    for some i of the group with x_i binary), give the primes; checked on the
    kernels' order (top digits first, then the digit above the in-block ones,
    then the in-block digits with the rest in one step) and on random
    orderings and partitions."""
    if kind == "dnf":
        tt = inputs.dnf(n, 8, 1, 4, 9400 + seed)
    else:
        tt = inputs.bernoulli(n, kind, 9400 + seed)
    M = np.zeros(3**n, dtype=bool)
    M[sorted(oracle.bitmap_to_set(n, oracle.enum_M(n, tt)))] = True
    _, O, _ = oracle.primes(n, tt)
    want = oracle.bitmap_to_set(n, O)
    rho = np.arange(3**n, dtype=np.int64)
    p3 = 3 ** np.arange(n, dtype=np.int64)
    digs = (rho[:, None] // p3[None, :]) % 3

    def staged(groups):
        S = M.copy()
        for g in groups:
            kill = np.zeros_like(S)
            for i in g:
                s = rho[digs[:, i] != 2]
                kill[s] |= S[s + (2 - digs[s, i]) * p3[i]]
            S &= ~kill
        return set(np.flatnonzero(S).tolist())

    # the kernels' order scaled down (0-based digits): the top group, the group
    # below it, one digit lo, then the digits under lo with those between lo
    # and the lower group in one step
    lo = (n - 4) // 2
    kernels = [[n - 2, n - 1], [n - 4, n - 3], [lo], list(range(lo)) + list(range(lo + 1, n - 4))]
    assert sorted(d for g in kernels for d in g) == list(range(n))
    assert staged(kernels) == want
    rng = random.Random(9400 + seed)
    for _ in range(6):
        order = list(range(n))
        rng.shuffle(order)
        cuts = sorted(rng.sample(range(1, n), rng.randint(0, n - 1)))
        groups = [order[a:b] for a, b in zip([0] + cuts, cuts + [n])]
        assert staged(groups) == want, groups
    assert want and len(want) < int(M.sum())


# ----------------------------------------------------------------------------
# the ranged ("streaming") O sweep and the block digests built on it


@pytest.mark.parametrize("n", list(range(0, 15)))
def test_ranged_sweep_matches_whole_and_bruteforce(n):
    """O evaluated one block of the top digits at a time, and on random
    unaligned ranges, gives the whole function's primes; for n <= 11 that list
    is also the brute force's (per-cube definitions of Sec. 2)."""
    tt = inputs.bernoulli(n, 0.85, 900 + n) if n % 2 else inputs.dnf(n, 3 * n + 1, 1, max(1, n // 2), 900 + n)
    M = oracle.enum_M(n, tt)
    whole, _ = oracle.extract(n, oracle.enum_O(n, M))
    if n <= 11:
        _, Ob = oracle.bruteforce(n, tt)
        ref, _ = oracle.extract(n, Ob)
        assert np.array_equal(whole, ref)
    top = min(n, 4)
    bs = 3 ** (n - top)
    parts = [oracle.primes_range(n, M, b * bs, (b + 1) * bs) for b in range(3**top)]
    assert np.array_equal(np.concatenate(parts), whole)
    rng = np.random.default_rng(n)
    for _ in range(8):
        a, b = sorted(int(v) for v in rng.integers(0, 3**n + 1, size=2))
        got = oracle.primes_range(n, M, a, b)
        assert np.array_equal(got, whole[(whole >= a) & (whole < b)]), (a, b)


@pytest.mark.parametrize("n,a,b", [(14, 5, 9), (13, 0, 13), (12, 6, 6)])
def test_ranged_sweep_closed_form(n, a, b):
    """Interval-symmetric f = [a <= |x| <= b]: its primes are the cubes with
    exactly a ones and b - a stars; the block-wise sweep lists exactly them."""
    M = oracle.enum_M(n, inputs.interval(n, a, b))
    bs = 3 ** (n - 4)
    got = np.concatenate([oracle.primes_range(n, M, k * bs, (k + 1) * bs) for k in range(81)])
    ref = sorted(r for r in _cubes_with(n, a, b - a))
    assert got.tolist() == ref


def _cubes_with(n, ones, stars):
    for pos in itertools.combinations(range(n), ones + stars):
        for sp in itertools.combinations(pos, stars):
            yield sum((2 if i in sp else 1) * 3**i for i in pos)


def test_block_digests_match_list_digests():
    """The digest writer's per-block form equals digests of the whole list,
    and a change to one prime changes exactly its block's line."""
    import sys
    sys.path.insert(0, GOLDEN)
    import make_block_digests as mbd

    for name, n in (("c3x", 12), ("c3x", 9)):
        spec = dict(inputs.CONFIGS["c3x_n21_dnf2000_noise"], n=n, seed=77 + n)
        tt = inputs.make(spec)
        M, O, lst = oracle.primes(n, tt)
        rows = mbd.block_digests(n, M)
        assert rows == mbd.digests_of_list(n, lst)
        assert sum(c for c, _ in rows) == lst.size
        bad = lst.copy()
        k = bad.size // 2
        bad = np.delete(bad, k)
        rows_bad = mbd.digests_of_list(n, bad)
        diff = [i for i in range(81) if rows_bad[i] != rows[i]]
        assert diff == [int(lst[k]) // 3 ** (n - 4)]


@pytest.mark.parametrize("config", ["c3x_n21_dnf2000_noise", "c3x_n22_dnf2000_noise",
                                    "c3x_n23_dnf2000_noise", "c3_n24_dnf2000_noise"])
def test_block_digest_files_well_formed(config):
    import sys
    sys.path.insert(0, GOLDEN)
    import make_block_digests as mbd

    if not os.path.exists(mbd.path_for(config)):
        pytest.skip("digest file not written yet")
    n, top, total, rows = mbd.read(config)
    assert n == inputs.CONFIGS[config]["n"] and top == 4
    assert len(rows) == 81 and sum(c for c, _ in rows) == total
    assert all(len(h) == 64 for _, h in rows)
    # the empty block's digest is the SHA-256 of no bytes
    import hashlib
    empty = hashlib.sha256(b"").hexdigest()
    assert all((c == 0) == (h == empty) for c, h in rows)
