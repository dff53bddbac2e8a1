"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a published
generator output, a plain definition (the product of the lifted inputs, the
tag relation of Eq. (1)), an identity between the two protocols, the
soundness of the MAC check, a special case that reduces to the single-value
check of Sec. 2.5, the closed-form costs of Sec. 3.4.3, or brute force with
Python integers on tiny shapes.
"""
import os

import numpy as np
import pytest

import oracle as O
from oracle import ref

R = 1 << 128
M64 = (1 << 64) - 1
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

SHAPES = [(1, 1, 1), (2, 3, 4), (4, 5, 3), (3, 1, 2), (5, 7, 1), (1, 6, 5), (6, 4, 9)]


def ints(a):
    return O.to_ints(a)


def lift(L, name):
    """sum of the two parties' shares, mod 2^128"""
    return (ints(L[name][0]) + ints(L[name][1])) % R


def dsum(L):
    return int(L.delta[0]) + int(L.delta[1])


def lifts_from_prng(L):
    """The dealt lifts recomputed directly from the generator definition."""
    M, K, N, seed, lid = L.M, L.K, L.N, L.seed, L.layer_id
    r0, r1 = L.r0, L.r1

    def d64(purpose, e):
        return ref.draw(seed, ref.stream(lid, purpose), e)

    def d128(purpose, e):
        return d64(purpose, 2 * e) | (d64(purpose, 2 * e + 1) << 64)

    X = np.array([[d64(1, i * K + k) for k in range(K)] for i in range(r0, r1)], dtype=object)
    Y = np.array([[d64(2, k * N + j) for j in range(N)] for k in range(K)], dtype=object)
    A = np.array([[d128(3, i * K + k) for k in range(K)] for i in range(r0, r1)], dtype=object)
    B = np.array([[d128(4, k * N + j) for j in range(N)] for k in range(K)], dtype=object)
    Rm = np.array([[d128(5, i * N + j) for j in range(N)] for i in range(r0, r1)], dtype=object)
    return X.reshape(r1 - r0, K), Y.reshape(K, N), A.reshape(r1 - r0, K), B.reshape(K, N), Rm.reshape(r1 - r0, N)


def omatmul(P, Q):
    return np.array([[sum(int(P[i, k]) * int(Q[k, j]) for k in range(P.shape[1])) % R
                      for j in range(Q.shape[1])] for i in range(P.shape[0])], dtype=object).reshape(
        P.shape[0], Q.shape[1])


@pytest.fixture(scope="module")
def built():
    O.build()


# ---------------------------------------------------------------- generator

def test_splitmix64_published_outputs(built):
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_state0.txt")) if l.startswith("0x")]
    gamma = 0x9E3779B97F4A7C15
    got = [O.mix64((n * gamma) & M64) for n in range(1, len(vals) + 1)]
    assert got == vals


def test_stream_draws_are_splitmix_outputs(built):
    # the i-th draw of a stream is output i+1 of SplitMix64 started at the stream key
    for seed, stream in [(0, 0), (1000, 0x10001), (2 ** 63 + 5, (7 << 16) | 0x32)]:
        key = O.lib().or_stream_key(seed, stream)
        state = key
        for i in range(5):
            state = (state + 0x9E3779B97F4A7C15) & M64
            assert O.draw(seed, stream, i) == O.mix64(state)
        assert key == O.mix64(seed ^ O.mix64(stream))


def test_python_generator_matches_c(built):
    for i in range(10):
        assert ref.draw(1001, (3 << 16) | 4, i) == O.draw(1001, (3 << 16) | 4, i)


# ---------------------------------------------------------------- dealer

@pytest.mark.parametrize("shape", SHAPES[:5])
def test_dealer_sharing_and_tags(built, shape):
    M, K, N = shape
    L = O.OracleLayer(M, K, N, seed=11, layer_id=3, key_seed=99).deal()
    X, Y, A, B, Rm = lifts_from_prng(L)
    key = dsum(L)
    assert int(L.delta[0]) < 2 ** 64 and int(L.delta[1]) < 2 ** 64
    C = omatmul(A, B)  # the triple: C~ = A~ B~ mod 2^{k+s}
    for name, v in [("X", X), ("Y", Y), ("A", A), ("B", B), ("C", C), ("R", Rm)]:
        assert (lift(L, name) == v).all(), name
        # Eq. (1): the tag shares sum to Delta~ * v~ mod 2^{k+s}
        assert (lift(L, "t" + name) == (key * v) % R).all(), name
    assert (X < 2 ** 64).all() and (Y < 2 ** 64).all()


def test_key_shares_one_zero_give_tags_equal_to_lifts(built):
    L = O.OracleLayer(3, 4, 2, seed=5, layer_id=1, key_seed=1)
    L.delta = np.array([1, 0], dtype=np.uint64)
    L.deal()
    for name in "XYABCR":
        assert (lift(L, "t" + name) == lift(L, name)).all()


# ---------------------------------------------------------------- online phase

@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("mode", [O.MODE_SPDZ2K, O.MODE_COMPACT])
def test_plain_definitions(built, shape, mode):
    M, K, N = shape
    L = O.run_layer(mode, M, K, N, seed=20 + M, layer_id=2, key_seed=77)
    X, Y, A, B, Rm = lifts_from_prng(L)
    XY = omatmul(X, Y)
    # Beaver correctness: the output shares reconstruct X~ Y~ mod 2^{k+s}
    Zt = lift(L, "Z")
    assert (Zt == XY).all()
    # and the value is the plain Z_{2^64} product
    Z64 = (np.array(Zt.reshape(-1) % 2 ** 64, dtype=np.uint64)).reshape(M, N)
    Xu = np.array(X.reshape(-1), dtype=np.uint64).reshape(M, K)
    Yu = np.array(Y.reshape(-1), dtype=np.uint64).reshape(K, N)
    with np.errstate(over="ignore"):
        assert (np.matmul(Xu, Yu) == Z64).all()
    # opened values
    assert (ints(L["E"]) == (X - A) % R).all()
    assert (ints(L["U"]) == (Y - B) % R).all()
    assert (ints(L["D"]) == (Rm - XY) % R).all()
    # tag relation on the output, both protocols
    assert (lift(L, "tZ") == (dsum(L) * XY) % R).all()


@pytest.mark.parametrize("shape", SHAPES)
def test_cross_mode_identities(built, shape):
    """CompactTag reaches the same authenticated output as SPDZ2k: identical value
    shares and opened matrices, equal tag sums, and per party the compact tag
    equals the SPDZ2k tag compressed by the same combiners."""
    M, K, N = shape
    S = O.run_layer(O.MODE_SPDZ2K, M, K, N, seed=31, layer_id=5, key_seed=4)
    C = O.run_layer(O.MODE_COMPACT, M, K, N, seed=31, layer_id=5, key_seed=4)
    for n in ("Z", "E", "U", "D"):
        assert (S[n] == C[n]).all(), n
    assert (lift(S, "tZ") == lift(C, "tZ")).all()
    chi = np.array([ref.draw(31, ref.stream(5, 0x30), j) for j in range(N)], dtype=object)
    for p in range(2):
        tZs = ints(S["tZ"][p]).reshape(M, N)
        expect = np.array([sum(int(tZs[i, j]) * int(chi[j]) for j in range(N)) % R for i in range(M)], dtype=object)
        assert (ints(C["tZc"][p]) == expect).all()
        # compact tag of D: [tD^c]_p = [tR]_p chi - [tZ]_p chi
        tRs = ints(C["tR"][p]).reshape(M, N)
        expD = np.array([sum((int(tRs[i, j]) - int(tZs[i, j])) * int(chi[j]) for j in range(N)) % R
                         for i in range(M)], dtype=object)
        assert (ints(C["tDc"][p]) == expD).all()
    # the compressed public matrices
    Dm = ints(C["D"]).reshape(M, N)
    assert (ints(C["Dc"]) == np.array([sum(int(Dm[i, j]) * int(chi[j]) for j in range(N)) % R
                                       for i in range(M)], dtype=object)).all()


@pytest.mark.parametrize("shape", SHAPES[:6])
@pytest.mark.parametrize("compact", [False, True])
def test_bruteforce_python_reference(built, shape, compact):
    M, K, N = shape
    mode = O.MODE_COMPACT if compact else O.MODE_SPDZ2K
    L = O.run_layer(mode, M, K, N, seed=41, layer_id=9, key_seed=8)
    S = {n: [ints(L[n][p]).reshape(L[n][p].shape[:-1]).tolist() for p in range(2)]
         for n in ("X", "tX", "A", "tA", "Y", "tY", "B", "tB", "C", "tC", "R", "tR")}
    delta = [int(L.delta[0]), int(L.delta[1])]
    out = ref.online_and_check(compact, M, K, N, 41, 9, delta, S)
    assert ints(L["E"]).reshape(M, K).tolist() == out["E"]
    assert ints(L["U"]).reshape(K, N).tolist() == out["U"]
    assert ints(L["D"]).reshape(M, N).tolist() == out["D"]
    for p in range(2):
        assert ints(L["Z"][p]).reshape(M, N).tolist() == out["Z"][p]
        assert ints(L["tZ"][p]).reshape(M, N).tolist() == out["tZ"][p]
        if compact:
            assert ints(L["tZc"][p]).tolist() == out["tZc"][p]
            assert ints(L["tDc"][p]).tolist() == out["tDc"][p]
    for w in range(3):
        for p in range(2):
            assert O.u128(L.cs[w, p]) == out["cs"][w][p], (w, p)


# ---------------------------------------------------------------- verification

@pytest.mark.parametrize("mode", [O.MODE_SPDZ2K, O.MODE_COMPACT])
def test_honest_runs_accept(built, mode):
    for seed in range(12):
        M, K, N = SHAPES[seed % len(SHAPES)]
        L = O.run_layer(mode, M, K, N, seed=100 + seed, layer_id=seed, key_seed=1000 + seed)
        assert L.cs_sums() == [0, 0, 0]
        assert L.accept()


TAMPER_TARGETS = [("X", 0), ("tX", 0), ("A", 2), ("tA", 2), ("Y", 1), ("tY", 1), ("B", 1), ("tB", 1),
                  ("C", 2), ("tC", 2), ("R", 2), ("tR", 2)]


@pytest.mark.parametrize("mode", [O.MODE_SPDZ2K, O.MODE_COMPACT])
@pytest.mark.parametrize("target", TAMPER_TARGETS)
@pytest.mark.parametrize("bit", [0, 31, 63])
def test_single_flipped_share_bit_aborts(built, mode, target, bit):
    """Flipping one bit below 2^k in one party's value or tag share makes the
    check that covers it fail (failure probability <= 2^{-s+log(s+1)}, Fig. 1
    and Theorem 1)."""
    name, w = target
    M, K, N = 3, 4, 5
    for party in (0, 1):
        L = O.OracleLayer(M, K, N, seed=7, layer_id=4, key_seed=3).deal()
        arr = L[name][party]
        flat = arr.reshape(-1, 2)
        idx = (5 * bit + 3) % flat.shape[0]
        flat[idx, 0] ^= np.uint64(1 << bit)
        L.online(mode).check(mode)
        sums = L.cs_sums()
        assert sums[w] != 0, (name, party, bit, sums)
        assert not L.accept()


def test_compact_check_with_unit_combiners_is_single_value_check(built):
    """With chi = e_j and chihat = e_i the compact check of D reduces to the
    single-value check of D_ij (Sec. 2.5): cs_p = -([tag D_ij]_p - D_ij [Delta]_p)."""
    M, K, N = 3, 4, 5
    L = O.run_layer(O.MODE_COMPACT, M, K, N, seed=3, layer_id=1, key_seed=2)
    D = L["D"]
    for i in range(M):
        for j in range(N):
            chi = np.zeros(N, dtype=np.uint64)
            chi[j] = 1
            chih = np.zeros(M, dtype=np.uint64)
            chih[i] = 1
            Dc = O.compress(D, chi)
            total = 0
            for p in range(2):
                tD = ((ints(L["tR"][p]) - ints(L["tZ"][p])) % R)
                tDc = O.compress(O.from_ints(tD), chi)
                cs = O.compact_cs(Dc, tDc, chih, int(L.delta[p]))
                single = (int(tD[i, j]) - O.u128(D[i, j]) * int(L.delta[p])) % R
                assert cs == (-single) % R
                total += cs
            assert total % R == 0


def test_batchrec_with_unit_combiner_is_single_value_check(built):
    M, K, N = 2, 3, 2
    L = O.run_layer(O.MODE_SPDZ2K, M, K, N, seed=9, layer_id=2, key_seed=5)
    E = L["E"]
    for e in range(M * K):
        chi = np.zeros(M * K, dtype=np.uint64)
        chi[e] = 1
        for p in range(2):
            tE = (ints(L["tX"][p]) - ints(L["tA"][p])) % R
            cs = O.batchrec_cs(E, O.from_ints(tE), chi, int(L.delta[p]))
            i, k = divmod(e, K)
            assert cs == (int(tE[i, k]) - O.u128(E[i, k]) * int(L.delta[p])) % R


def test_rows_ranges_compose(built):
    """Running rows [r0, r1) pieces reproduces the full run and the check-value
    shares add up (this is how full-size layers are sampled)."""
    M, K, N = 7, 5, 4
    for mode in (O.MODE_SPDZ2K, O.MODE_COMPACT):
        full = O.run_layer(mode, M, K, N, seed=13, layer_id=6, key_seed=21)
        cuts = [0, 2, 3, 7]
        cs = [[0, 0], [0, 0], [0, 0]]
        for a, b in zip(cuts[:-1], cuts[1:]):
            part = O.run_layer(mode, M, K, N, seed=13, layer_id=6, key_seed=21, r0=a, r1=b)
            for n in ("E", "tX"):
                sl = full[n][a:b] if n == "E" else full[n][:, a:b]
                assert (part[n] == sl).all()
            for n in ("Z", "tZ"):
                assert (part[n] == full[n][:, a:b]).all()
            assert (part["D"] == full["D"][a:b]).all()
            if mode == O.MODE_COMPACT:
                assert (part["tDc"] == full["tDc"][:, a:b]).all()
            for w in (0, 2):
                for p in range(2):
                    cs[w][p] += O.u128(part.cs[w, p])
            assert (part["U"] == full["U"]).all()
        for w in (0, 2):
            for p in range(2):
                assert cs[w][p] % R == O.u128(full.cs[w, p])


# ---------------------------------------------------------------- readings

def test_literal_k_plus_2s_check_rejects_honest_runs(built):
    """Documents the reading of Fig. 7 verification steps 4-6: evaluated mod
    2^{k+2s} on the 128-bit shares, the honest compact check fails most of the
    time, while mod 2^{k+s} it always passes."""
    R192 = 1 << 192
    fails = 0
    trials = 40
    for t in range(trials):
        L = O.run_layer(O.MODE_COMPACT, 3, 2, 2, seed=500 + t, layer_id=1, key_seed=600 + t)
        assert L.accept()
        chih = [ref.draw(500 + t, ref.stream(1, 0x31), i) for i in range(3)]
        s = 0
        for p in range(2):
            Dc = ints(L["Dc"])
            tDc = ints(L["tDc"][p])
            for i in range(3):
                cs_i = ((int(L.delta[p]) * int(Dc[i])) % R) * chih[i] - int(tDc[i]) * chih[i]
                s += cs_i
        fails += (s % R192) != 0
    assert fails > trials // 2


def test_party1_only_key_term_breaks_tag_relation(built):
    """Documents the reading of Fig. 2 step 3: if only one party adds its key
    share times E*U, the tag shares no longer sum to Delta~ * Z~."""
    M, K, N = 3, 4, 2
    L = O.run_layer(O.MODE_SPDZ2K, M, K, N, seed=17, layer_id=2, key_seed=19)
    EU = omatmul(ints(L["E"]).reshape(M, K), ints(L["U"]).reshape(K, N))
    literal = (ints(L["tZ"][0]) + ints(L["tZ"][1]) - int(L.delta[1]) * EU) % R
    assert not (literal == (dsum(L) * lift(L, "Z")) % R).any()


# ---------------------------------------------------------------- costs

@pytest.mark.parametrize("shape", SHAPES + [(8, 16, 32), (33, 7, 2)])
def test_tag_multiplication_counts_match_closed_forms(built, shape):
    M, K, N = shape
    S = O.run_layer(O.MODE_SPDZ2K, M, K, N, seed=1, layer_id=1, key_seed=1)
    C = O.run_layer(O.MODE_COMPACT, M, K, N, seed=1, layer_id=1, key_seed=1)
    for p in range(2):
        assert int(S.tag_mults[p]) == O.spdz2k_tag_mults(M, K, N)
        assert int(C.tag_mults[p]) == O.compact_tag_mults(M, K, N)


def test_paper_384x_example():
    kv = dict(l.strip().split("=") for l in open(os.path.join(GOLDEN, "paper_op_counts.txt"))
              if "=" in l and not l.startswith("#"))
    T1, T2, T3 = int(kv["T1"]), int(kv["T2"]), int(kv["T3"])
    ratio = O.spdz2k_tag_mults(T1, T2, T3) / O.compact_tag_mults(T1, T2, T3)
    assert round(ratio) == int(kv["printed_ratio"])
    assert abs(ratio - 384.08) < 0.01


# ---------------------------------------------------------------- truncation (f > 0)

def signed64(v):
    v = int(v) % (1 << 64)
    return v - (1 << 64) if v >= 1 << 63 else v


@pytest.mark.parametrize("f", [1, 13, 40, 63])
def test_truncation_dealer_mask(built, f):
    """The dealt R^f is (R mod 2^k) / 2^f as an integer, authenticated (Eq. (1))."""
    L = O.OracleLayer(5, 3, 7, 77, 4, 9, f=f).deal()
    R_k = lift(L, "R") % (1 << 64)
    Rf = lift(L, "Rf")
    assert np.array_equal((Rf % (1 << 64)).astype(object), (R_k // (1 << f)).astype(object))
    assert np.array_equal(lift(L, "tRf"), (dsum(L) * Rf) % R)
    # the upper limb of the lift is a fresh uniform draw (not a copy of R's)
    assert any(int(v) >> 64 != int(w) >> 64 for v, w in zip(Rf.ravel(), lift(L, "R").ravel()))


@pytest.mark.parametrize("shape", SHAPES)
def test_truncation_tag_relation_and_modes(built, shape):
    """Both protocols output the same truncated shares and tags (Figs. 3 and 6
    use the same formulas), whose tags satisfy Eq. (1) with Delta~."""
    M, K, N = shape
    outs = {}
    for mode in (O.MODE_SPDZ2K, O.MODE_COMPACT):
        L = O.run_layer(mode, M, K, N, seed=91, layer_id=3, key_seed=5, f=17, in_bits=20)
        assert L.accept()
        assert np.array_equal(lift(L, "tZf"), (dsum(L) * lift(L, "Zf")) % R)
        outs[mode] = L
    for n in ("Zf", "tZf"):
        for p in range(2):
            assert np.array_equal(outs[0][n][p], outs[1][n][p]), (n, p)


@pytest.mark.parametrize("f", [8, 13, 24])
def test_truncation_accuracy(built, f):
    """With signed 16-bit inputs the product z = X Y is small, and the
    truncated output reconstructs to floor(z / 2^f) or one more, mod 2^64,
    for every element where R mod 2^64 - z does not leave [0, 2^64) -- the
    correctness condition of truncation by a random mask (Sec. 3.4.2)."""
    M, K, N = 24, 40, 9
    for seed in (3, 4):
        L = O.run_layer(O.MODE_COMPACT, M, K, N, seed=seed, layer_id=12, key_seed=2, f=f, in_bits=16)
        X = [[signed64(v) for v in row] for row in lift(L, "X").tolist()]
        Y = [[signed64(v) for v in row] for row in lift(L, "Y").tolist()]
        assert max(abs(v) for row in X for v in row) < 1 << 15
        R_k = lift(L, "R") % (1 << 64)
        Zf = lift(L, "Zf") % (1 << 64)
        wraps = 0
        for i in range(M):
            for j in range(N):
                z = sum(X[i][k] * Y[k][j] for k in range(K))
                if not 0 <= int(R_k[i, j]) - z < 1 << 64:
                    wraps += 1
                    continue
                err = (int(Zf[i, j]) - (z >> f)) % (1 << 64)
                assert err in (0, 1), (i, j, err)
        assert wraps <= 1


def test_truncation_mask_is_not_covered_by_the_layer_check(built):
    """A flipped bit in a share of R^f leaves this layer's check accepting (the
    truncated mask is only consumed by the outputs) but breaks the tag
    relation of the output, which the next check that opens it catches."""
    L = O.OracleLayer(4, 6, 5, 19, 2, 3, f=9).deal()
    L["Rf"][1][2, 3, 0] ^= np.uint64(1 << 7)
    L.online(O.MODE_COMPACT).check(O.MODE_COMPACT)
    assert L.accept()
    assert not np.array_equal(lift(L, "tZf"), (dsum(L) * lift(L, "Zf")) % R)


@pytest.mark.parametrize("compact", [False, True])
def test_truncation_bruteforce(built, compact):
    M, K, N = 3, 4, 5
    mode = O.MODE_COMPACT if compact else O.MODE_SPDZ2K
    L = O.run_layer(mode, M, K, N, seed=44, layer_id=6, key_seed=8, f=11)
    names = ("X", "tX", "A", "tA", "Y", "tY", "B", "tB", "C", "tC", "R", "tR", "Rf", "tRf")
    S = {n: [ints(L[n][p]).reshape(L[n][p].shape[:-1]).tolist() for p in range(2)] for n in names}
    delta = [int(L.delta[0]), int(L.delta[1])]
    out = ref.online_and_check(compact, M, K, N, 44, 6, delta, S, f=11)
    for p in range(2):
        assert ints(L["Zf"][p]).reshape(M, N).tolist() == out["Zf"][p]
        assert ints(L["tZf"][p]).reshape(M, N).tolist() == out["tZf"][p]


# ---------------------------------------------------------------- k = s = 32 (shares in Z_{2^64})

R64 = 1 << 64
M32 = (1 << 32) - 1


def lift64(L, name):
    return (ints(L[name][0]) + ints(L[name][1])) % R64


def test_k32_key_shares_and_dealer(built):
    """Key shares are the key draws mod 2^32; every dealt object's shares sum to
    its lift recomputed from the generator (inputs mod 2^32, masks mod 2^64)
    and its tag shares to Delta~ times the lift, mod 2^64."""
    d = O.key_shares(7, 32)
    for p in range(2):
        assert int(d[p]) == ref.draw(7, ref.stream(0xFFFF, 0x40 + p), 0) & M32
    M, K, N, seed, lid = 3, 4, 5, 23, 6
    L = O.OracleLayer(M, K, N, seed, lid, 7, kbits=32).deal()
    ds = dsum(L)
    assert ds < 1 << 33
    d64 = lambda purpose, e: ref.draw(seed, ref.stream(lid, purpose), e)
    X = np.array([[d64(1, i * K + k) & M32 for k in range(K)] for i in range(M)], dtype=object)
    A = np.array([[d64(3, 2 * (i * K + k)) for k in range(K)] for i in range(M)], dtype=object)
    Y = np.array([[d64(2, k * N + j) & M32 for j in range(N)] for k in range(K)], dtype=object)
    B = np.array([[d64(4, 2 * (k * N + j)) for j in range(N)] for k in range(K)], dtype=object)
    assert np.array_equal(lift64(L, "X"), X) and np.array_equal(lift64(L, "A"), A)
    assert np.array_equal(lift64(L, "Y"), Y) and np.array_equal(lift64(L, "B"), B)
    C = np.array([[sum(A[i, k] * B[k, j] for k in range(K)) % R64 for j in range(N)] for i in range(M)],
                 dtype=object)
    assert np.array_equal(lift64(L, "C"), C)
    for n in ("X", "A", "Y", "B", "C", "R"):
        assert np.array_equal(lift64(L, "t" + n), (ds * lift64(L, n)) % R64), n
        assert not L[n][1][..., 1].any()   # upper limb stays zero


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("mode", [O.MODE_SPDZ2K, O.MODE_COMPACT])
def test_k32_plain_definitions(built, shape, mode):
    M, K, N = shape
    L = O.run_layer(mode, M, K, N, seed=31, layer_id=4, key_seed=9, kbits=32)
    X, Y = lift64(L, "X"), lift64(L, "Y")
    Z = lift64(L, "Z")
    assert np.array_equal(Z, omatmul(X, Y) % R64)
    # Z mod 2^32 is the wrapping uint32 product of the inputs
    z32 = (X.astype(np.uint64).astype(np.uint32).astype(np.uint64) @
           Y.astype(np.uint64).astype(np.uint32).astype(np.uint64)) & np.uint64(M32)
    assert np.array_equal((Z % (1 << 32)).astype(np.uint64), z32)
    assert np.array_equal(lift64(L, "tZ"), (dsum(L) * Z) % R64)
    assert L.accept()


@pytest.mark.parametrize("shape", SHAPES[:5])
def test_k32_cross_mode_identity(built, shape):
    """Per party, the compact tag equals the SPDZ2k tag compressed by chi (mod 2^64)."""
    M, K, N = shape
    Ls = O.run_layer(O.MODE_SPDZ2K, M, K, N, seed=12, layer_id=2, key_seed=3, kbits=32)
    Lc = O.run_layer(O.MODE_COMPACT, M, K, N, seed=12, layer_id=2, key_seed=3, kbits=32)
    chi = [ref.draw(12, ref.stream(2, 0x30), j) & M32 for j in range(N)]
    for p in range(2):
        tz = ints(Ls["tZ"][p]).reshape(M, N)
        want = [sum(int(tz[i, j]) * chi[j] for j in range(N)) % R64 for i in range(M)]
        assert ints(Lc["tZc"][p]).tolist() == want
        assert np.array_equal(Ls["Z"][p], Lc["Z"][p])


@pytest.mark.parametrize("mode", [O.MODE_SPDZ2K, O.MODE_COMPACT])
@pytest.mark.parametrize("target,bit", [("X", 0), ("tA", 31), ("Y", 17), ("tB", 5), ("C", 20), ("tR", 31)])
def test_k32_single_flipped_share_bit_aborts(built, mode, target, bit):
    L = O.OracleLayer(4, 5, 6, 61, 8, 2, kbits=32).deal()
    L[target][1][1, 2, 0] ^= np.uint64(1 << bit)
    L.online(mode).check(mode)
    assert not L.accept()


@pytest.mark.parametrize("compact", [False, True])
def test_k32_bruteforce(built, compact):
    M, K, N = 3, 4, 5
    mode = O.MODE_COMPACT if compact else O.MODE_SPDZ2K
    L = O.run_layer(mode, M, K, N, seed=45, layer_id=7, key_seed=8, f=9, kbits=32)
    names = ("X", "tX", "A", "tA", "Y", "tY", "B", "tB", "C", "tC", "R", "tR", "Rf", "tRf")
    S = {n: [ints(L[n][p]).reshape(L[n][p].shape[:-1]).tolist() for p in range(2)] for n in names}
    delta = [int(L.delta[0]), int(L.delta[1])]
    out = ref.online_and_check(compact, M, K, N, 45, 7, delta, S, f=9, kbits=32)
    for p in range(2):
        assert ints(L["Z"][p]).reshape(M, N).tolist() == out["Z"][p]
        assert ints(L["tZ"][p]).reshape(M, N).tolist() == out["tZ"][p]
        assert ints(L["Zf"][p]).reshape(M, N).tolist() == out["Zf"][p]
    for w in range(3):
        for p in range(2):
            assert O.u128(L.cs[w, p]) == out["cs"][w][p], (w, p)


@pytest.mark.parametrize("f", [4, 10])
def test_k32_truncation_accuracy(built, f):
    M, K, N = 12, 20, 7
    L = O.run_layer(O.MODE_COMPACT, M, K, N, seed=5, layer_id=13, key_seed=2, f=f, in_bits=8, kbits=32)
    sg = lambda v: (int(v) % (1 << 32)) - (1 << 32) * ((int(v) % (1 << 32)) >= 1 << 31)
    X = [[sg(v) for v in row] for row in lift64(L, "X").tolist()]
    Y = [[sg(v) for v in row] for row in lift64(L, "Y").tolist()]
    R_k = lift64(L, "R") % (1 << 32)
    Zf = lift64(L, "Zf") % (1 << 32)
    assert np.array_equal(lift64(L, "tZf"), (dsum(L) * lift64(L, "Zf")) % R64)
    for i in range(M):
        for j in range(N):
            z = sum(X[i][k] * Y[k][j] for k in range(K))
            if 0 <= int(R_k[i, j]) - z < 1 << 32:
                assert (int(Zf[i, j]) - (z >> f)) % (1 << 32) in (0, 1)


# ---------------------------------------------------------------- compression along M

def transposed_layer(L, kbits=64):
    """The product Z^T = Y^T X^T as a layer of its own (M' = N, K' = K, N' = M)
    holding L's dealt shares transposed: X' = Y^T, A' = B^T, Y' = X^T, B' = A^T,
    C' = C^T, R' = R^T, each with its tags, same seed, layer id and key."""
    T = O.OracleLayer(L.N, L.K, L.M, L.seed, L.layer_id, L.key_seed, kbits=kbits, f=L.f)
    pairs = {"X": "Y", "tX": "tY", "A": "B", "tA": "tB", "Y": "X", "tY": "tX", "B": "A", "tB": "tA",
             "C": "C", "tC": "tC", "R": "R", "tR": "tR", "Rf": "Rf", "tRf": "tRf"}
    for dst, src in pairs.items():
        for p in range(2):
            T[dst][p][...] = np.ascontiguousarray(np.swapaxes(L[src][p], 0, 1))
    return T


CMP_SHAPES = [(1, 1, 1), (4, 5, 3), (6, 4, 9), (9, 2, 1), (5, 7, 1), (3, 8, 2)]


@pytest.mark.parametrize("kbits", [64, 32])
@pytest.mark.parametrize("shape", CMP_SHAPES)
def test_compress_along_m_is_compress_along_n_of_the_transpose(built, shape, kbits):
    """Compressing along M is the compact tag of the transposed product
    (Z^T = Y^T X^T, Eq. (5) multiplied from the left): the compressed vectors,
    the compact tags and the check of D equal those of the compression along N
    of the transposed layer, whose combiners chi (length M) and chihat (length N)
    are the same draws."""
    M, K, N = shape
    L = O.OracleLayer(M, K, N, 61, 3, 9, kbits=kbits, compress=1).deal()
    T = transposed_layer(L, kbits)
    L.online(O.MODE_COMPACT).check(O.MODE_COMPACT)
    T.online(O.MODE_COMPACT).check(O.MODE_COMPACT)
    assert L.accept() and T.accept()
    sw = lambda a: np.ascontiguousarray(np.swapaxes(a, 0, 1))
    assert (T["E"] == sw(L["U"])).all() and (T["U"] == sw(L["E"])).all() and (T["D"] == sw(L["D"])).all()
    for p in range(2):
        assert (T["Z"][p] == sw(L["Z"][p])).all() and (T["tZ"][p] == sw(L["tZ"][p])).all()
    assert (T["Uc"] == L["Ec"]).all()
    for n in ("Dc", "EUc"):
        assert (T[n] == L[n]).all(), n
    for p in range(2):
        assert (T["tBc"][p] == L["tAc"][p]).all()
        for n in ("tCc", "tRc", "tZc", "tDc"):
            assert (T[n][p] == L[n][p]).all(), (n, p)
        assert (T.cs[2, p] == L.cs[2, p]).all()
    assert list(L.tag_mults) == list(T.tag_mults) == [O.compact_tag_mults(M, K, N, 1)] * 2


@pytest.mark.parametrize("shape", CMP_SHAPES)
def test_compress_along_m_tag_relation(built, shape):
    """Per the MAC relation, the compact tag shares of chi^T Z sum to
    Delta~ chi^T Z~, those of chi^T D~ to Delta~ chi^T D~, and the value
    shares, tags and opened matrices are those of the compression along N."""
    M, K, N = shape
    L = O.run_layer(O.MODE_COMPACT, M, K, N, 71, 4, 6, compress=1)
    C = O.run_layer(O.MODE_COMPACT, M, K, N, 71, 4, 6)
    for n in ("Z", "tZ", "E", "U", "D"):
        assert (L[n] == C[n]).all(), n
    chi = [ref.draw(71, ref.stream(4, 0x30), i) for i in range(M)]
    Zt, Dt = lift(L, "Z").reshape(M, N), ints(L["D"]).reshape(M, N)
    cZ = [sum(chi[i] * int(Zt[i, j]) for i in range(M)) % R for j in range(N)]
    cD = [sum(chi[i] * int(Dt[i, j]) for i in range(M)) % R for j in range(N)]
    assert ints(L["Dc"]).tolist() == cD
    assert lift(L, "tZc").tolist() == [dsum(L) * v % R for v in cZ]
    assert lift(L, "tDc").tolist() == [dsum(L) * v % R for v in cD]
    Et = ints(L["E"]).reshape(M, K)
    assert ints(L["Ec"]).tolist() == [sum(chi[i] * int(Et[i, k]) for i in range(M)) % R for k in range(K)]


@pytest.mark.parametrize("target", [("tC", 2), ("tR", 2), ("R", 2), ("C", 2), ("tA", 0), ("tB", 1)])
@pytest.mark.parametrize("bit", [0, 40])
def test_compress_along_m_flipped_bit_aborts(built, target, bit):
    name, w = target
    M, K, N = 5, 4, 3
    for party in (0, 1):
        L = O.OracleLayer(M, K, N, seed=8, layer_id=6, key_seed=3, compress=1).deal()
        flat = L[name][party].reshape(-1, 2)
        flat[(7 * bit + 2) % flat.shape[0], 0] ^= np.uint64(1 << bit)
        L.online(O.MODE_COMPACT).check(O.MODE_COMPACT)
        assert L.cs_sums()[w] != 0 and not L.accept(), (name, party, bit)


def test_compressed_dimension_choice():
    """The count of Sec. 3.4.3 with M and N exchanged is smaller exactly when
    M > N: the classifier at batch 1 compresses along M (1.5x fewer
    multiplications), the encoder products along N."""
    assert O.cheaper_compress(4096, 25088, 1) == 1
    assert O.compact_tag_mults(4096, 25088, 1) / O.compact_tag_mults(4096, 25088, 1, 1) > 1.49
    assert O.cheaper_compress(128, 768, 2304) == 0 and O.cheaper_compress(64, 576, 3136) == 0
    assert O.cheaper_compress(512, 4608, 49) == 1 and O.cheaper_compress(7, 5, 7) == 0
    for M, K, N in [(3, 9, 2), (2, 9, 3), (5, 1, 5), (1, 1, 8)]:
        a, b = O.compact_tag_mults(M, K, N, 0), O.compact_tag_mults(M, K, N, 1)
        assert (b < a) == (M > N) and (a == b) == (M == N)


def test_compress_along_m_needs_all_rows(built):
    with pytest.raises(ValueError):
        O.OracleLayer(6, 3, 2, 1, 1, 1, r0=2, r1=4, compress=1)


# ---------------------------------------------------------------- convolution (Eq. (4))

CONVS = [  # (C_out, (C, H, W, k, stride, pad))
    (3, (2, 5, 5, 3, 1, 1)), (2, (3, 4, 6, 3, 2, 0)), (4, (1, 7, 5, 3, 2, 1)), (2, (2, 3, 3, 1, 1, 0)),
    (3, (2, 6, 4, 2, 2, 1))]


def conv_dims(cout, g):
    C, H, W, k, s, p = g
    Ho, Wo = (H + 2 * p - k) // s + 1, (W + 2 * p - k) // s + 1
    return cout, C * k * k, Ho * Wo, Ho, Wo


@pytest.mark.parametrize("cout,g", CONVS)
@pytest.mark.parametrize("mode", [O.MODE_SPDZ2K, O.MODE_COMPACT])
def test_conv_output_is_the_direct_convolution(built, cout, g, mode):
    """Sum_p [Z]_p is the convolution of the lifted weights with the lifted
    input, computed by its defining sum over channels and kernel taps (no
    im2col), mod 2^128; the tags satisfy Eq. (1)."""
    C, H, W, k, s, p = g
    M, K, N, Ho, Wo = conv_dims(cout, g)
    L = O.run_layer(mode, M, K, N, 13, 6, 5, conv=g)
    Wt = lift(L, "X").reshape(cout, C, k, k)
    In = lift(L, "Y").reshape(C, H, W)
    Z = lift(L, "Z").reshape(cout, Ho, Wo)
    for o in range(cout):
        for y in range(Ho):
            for x in range(Wo):
                acc = 0
                for c in range(C):
                    for dy in range(k):
                        for dx in range(k):
                            iy, ix = y * s + dy - p, x * s + dx - p
                            if 0 <= iy < H and 0 <= ix < W:
                                acc += int(Wt[o, c, dy, dx]) * int(In[c, iy, ix])
                assert int(Z[o, y, x]) == acc % R, (o, y, x)
    assert (lift(L, "tZ") == (dsum(L) * lift(L, "Z")) % R).all()
    assert L.accept()


@pytest.mark.parametrize("cout,g", CONVS[:3])
def test_conv_matches_torch_conv2d(built, cout, g):
    """With 6-bit signed inputs the product mod 2^64 equals torch's float64
    conv2d (exact at these magnitudes): pins the im2col ordering of Eq. (4)
    against a library convolution."""
    import torch
    C, H, W, k, s, p = g
    M, K, N, Ho, Wo = conv_dims(cout, g)
    L = O.run_layer(O.MODE_COMPACT, M, K, N, 17, 2, 3, in_bits=6, conv=g)
    sg = lambda v: (int(v) % 2 ** 64) - 2 ** 64 * ((int(v) % 2 ** 64) >= 2 ** 63)
    Wt = torch.tensor([[sg(v) for v in row] for row in lift(L, "X").tolist()], dtype=torch.float64)
    In = torch.tensor([[sg(v) for v in row] for row in lift(L, "Y").tolist()], dtype=torch.float64)
    ref = torch.nn.functional.conv2d(In.reshape(1, C, H, W), Wt.reshape(cout, C, k, k), stride=s, padding=p)
    got = [[sg(v) for v in row] for row in lift(L, "Z").tolist()]
    assert torch.equal(ref.reshape(cout, Ho * Wo), torch.tensor(got, dtype=torch.float64))


@pytest.mark.parametrize("cout,g", CONVS)
@pytest.mark.parametrize("mode", [O.MODE_SPDZ2K, O.MODE_COMPACT])
def test_conv_equals_the_explicit_product(built, cout, g, mode):
    """A convolution layer is the plain product on the im2col matrices of its
    input shares, mask shares and tags: the same output shares, tags, opened
    E and D, compact vectors and checks of E and D; only U is opened (and
    checked) on the input's shape, and its im2col is the product's U."""
    M, K, N, Ho, Wo = conv_dims(cout, g)
    Lc = O.OracleLayer(M, K, N, 23, 8, 4, conv=g).deal()
    Lx = O.OracleLayer(M, K, N, 23, 8, 4).deal()
    for n in ("Y", "tY", "B", "tB"):
        for q in range(2):
            Lx[n][q][...] = O.im2col(Lc, Lc[n][q])
    for n in ("X", "tX", "A", "tA", "C", "tC", "R", "tR"):   # C~ = A~ im2col(B~) in both
        assert (Lx[n] == Lc[n]).all() if n in ("X", "tX", "A", "tA", "R", "tR") else True
        Lx[n][...] = Lc[n]
    Lc.online(mode).check(mode)
    Lx.online(mode).check(mode)
    assert Lc.accept() and Lx.accept()
    for n in ("Z", "tZ", "E", "D"):
        assert (Lc[n] == Lx[n]).all(), n
    assert (O.im2col(Lc, Lc["U"]) == Lx["U"]).all()
    if mode == O.MODE_COMPACT:
        for n in ("Uc", "tBc", "Dc", "EUc", "tCc", "tRc", "tZc", "tDc"):
            assert (Lc[n] == Lx[n]).all(), n
    for w in (0, 2):
        assert (Lc.cs[w] == Lx.cs[w]).all()
    assert list(Lc.tag_mults) == list(Lx.tag_mults)


@pytest.mark.parametrize("cout,g", CONVS)
def test_conv_compression_is_a_correlation(built, cout, g):
    """Compressing the im2col matrix along N is a k x k correlation of the
    input with the combiners laid out as an Ho x Wo image:
    U^c[(c, dy, dx)] = sum_{y, x} chi[y Wo + x] U[c, y s + dy - p, x s + dx - p]."""
    C, H, W, k, s, p = g
    M, K, N, Ho, Wo = conv_dims(cout, g)
    L = O.run_layer(O.MODE_COMPACT, M, K, N, 29, 3, 2, conv=g)
    chi = [ref.draw(29, ref.stream(3, 0x30), j) for j in range(N)]
    U = ints(L["U"]).reshape(C, H, W)
    for q in range(2):
        tB = ints(L["tB"][q]).reshape(C, H, W)
        for c in range(C):
            for dy in range(k):
                for dx in range(k):
                    su = st = 0
                    for y in range(Ho):
                        for x in range(Wo):
                            iy, ix = y * s + dy - p, x * s + dx - p
                            if 0 <= iy < H and 0 <= ix < W:
                                su += chi[y * Wo + x] * int(U[c, iy, ix])
                                st += chi[y * Wo + x] * int(tB[c, iy, ix])
                    kk = (c * k + dy) * k + dx
                    assert O.u128(L["Uc"][kk]) == su % R
                    assert O.u128(L["tBc"][q][kk]) == st % R


@pytest.mark.parametrize("target", ["Y", "tY", "B", "tB"])
@pytest.mark.parametrize("mode", [O.MODE_SPDZ2K, O.MODE_COMPACT])
def test_conv_flipped_input_bit_aborts_the_check_of_u(built, target, mode):
    """U is opened and checked on the input's elements: one flipped bit of an
    input or mask share (value or tag) fails the check of U."""
    cout, g = CONVS[0]
    M, K, N, Ho, Wo = conv_dims(cout, g)
    for party in (0, 1):
        L = O.OracleLayer(M, K, N, 31, 5, 6, conv=g).deal()
        L[target][party].reshape(-1, 2)[7, 0] ^= np.uint64(1 << 21)
        L.online(mode).check(mode)
        assert L.cs_sums()[1] != 0 and not L.accept(), (target, party)


@pytest.mark.parametrize("kbits", [64, 32])
def test_conv_with_compression_along_m_and_k32(built, kbits):
    cout, g = 12, (2, 4, 4, 3, 2, 1)     # M = 12 > N = 4: the cheaper compression is along M
    M, K, N, Ho, Wo = conv_dims(cout, g)
    assert O.cheaper_compress(M, K, N) == 1
    L = O.run_layer(O.MODE_COMPACT, M, K, N, 37, 7, 8, kbits=kbits, compress=1, conv=g)
    Ln = O.run_layer(O.MODE_COMPACT, M, K, N, 37, 7, 8, kbits=kbits, compress=0, conv=g)
    assert L.accept() and Ln.accept()
    for n in ("Z", "tZ", "D", "U"):
        assert (L[n] == Ln[n]).all()


def test_conv_geometry_is_validated(built):
    with pytest.raises(ValueError):
        O.OracleLayer(3, 18, 24, 1, 1, 1, conv=(2, 5, 5, 3, 1, 1))


# ---------------------------------------------------------------- n parties

def nlift(L, name):
    """sum of all parties' shares, mod 2^128"""
    return sum(ints(L[name][p]) for p in range(L.parties)) % R


@pytest.mark.parametrize("parties", [3, 4, 5])
@pytest.mark.parametrize("shape", [(2, 3, 4), (5, 7, 1), (6, 4, 9)])
@pytest.mark.parametrize("mode", [O.MODE_SPDZ2K, O.MODE_COMPACT])
def test_parties_plain_definitions(built, parties, shape, mode):
    """With n parties the shares of every dealt value sum to its lift (the
    lifts do not depend on n), sum_p [Z]_p = X~ Y~, the tags of Z sum to
    Delta~ Z~ with Delta~ the sum of the n key shares, and the check accepts."""
    M, K, N = shape
    L = O.run_layer(mode, M, K, N, 20 + M, 2, 77, parties=parties)
    X, Y, A, B, Rm = lifts_from_prng(L)
    assert (nlift(L, "X") == X).all() and (nlift(L, "Y") == Y).all() and (nlift(L, "A") == A).all()
    assert (nlift(L, "B") == B).all() and (nlift(L, "R") == Rm).all()
    dn = sum(int(v) for v in L.delta)
    assert len(L.delta) == parties
    assert list(L.delta[:2]) == list(O.key_shares(77))          # party keys do not depend on n
    for n in ("X", "A", "C", "R"):
        assert (nlift(L, "t" + n) == (dn * nlift(L, n)) % R).all(), n
    XY = omatmul(X, Y)
    assert (nlift(L, "Z") == XY).all()
    assert (ints(L["D"]) == (Rm - XY) % R).all()
    assert (nlift(L, "tZ") == (dn * XY) % R).all()
    assert L.accept()


@pytest.mark.parametrize("parties", [3, 5])
def test_parties_dealer_streams(built, parties):
    """Party p < n - 1 draws its value and tag shares from the streams of
    purpose 0x10 / 0x20 + object + 256 p; the last party completes the sums
    (with n = 2 this is the two-party dealer)."""
    M, K, N = 2, 3, 2
    L = O.OracleLayer(M, K, N, seed=11, layer_id=3, key_seed=9, parties=parties).deal()
    for p in range(parties - 1):
        for i in range(M):
            for k in range(K):
                e = i * K + k
                d = lambda purpose: (ref.draw(11, ref.stream(3, purpose), 2 * e)
                                     | (ref.draw(11, ref.stream(3, purpose), 2 * e + 1) << 64))
                assert O.u128(L["A"][p][i, k]) == d(0x10 + 3 + 256 * p)
                assert O.u128(L["tA"][p][i, k]) == d(0x20 + 3 + 256 * p)


@pytest.mark.parametrize("parties", [3, 4])
def test_parties_cross_mode_identity(built, parties):
    """Per party, the compact tag equals the SPDZ2k tag compressed by chi."""
    M, K, N = 4, 5, 3
    S = O.run_layer(O.MODE_SPDZ2K, M, K, N, 31, 5, 4, parties=parties)
    C = O.run_layer(O.MODE_COMPACT, M, K, N, 31, 5, 4, parties=parties)
    chi = [ref.draw(31, ref.stream(5, 0x30), j) for j in range(N)]
    for n in ("Z", "E", "U", "D"):
        assert (S[n] == C[n]).all(), n
    for p in range(parties):
        tZs = ints(S["tZ"][p]).reshape(M, N)
        expect = [sum(int(tZs[i, j]) * chi[j] for j in range(N)) % R for i in range(M)]
        assert ints(C["tZc"][p]).tolist() == expect, p


@pytest.mark.parametrize("parties", [2, 3, 5])
def test_parties_tag_work_per_party_is_unchanged(built, parties):
    """The tag multiplications of each party are the two-party closed forms of
    Sec. 3.4.3 for any number of parties (Appendix: CompactTag scales with
    parties)."""
    M, K, N = 6, 4, 9
    for mode in (O.MODE_SPDZ2K, O.MODE_COMPACT):
        L = O.run_layer(mode, M, K, N, 3, 1, 2, parties=parties)
        want = O.spdz2k_tag_mults(M, K, N) if mode == O.MODE_SPDZ2K else O.compact_tag_mults(M, K, N)
        assert list(L.tag_mults) == [want] * parties


@pytest.mark.parametrize("parties", [3, 5])
@pytest.mark.parametrize("mode", [O.MODE_SPDZ2K, O.MODE_COMPACT])
@pytest.mark.parametrize("target", [("X", 0), ("tA", 0), ("Y", 1), ("tB", 1), ("C", 2), ("tR", 2)])
def test_parties_flipped_bit_aborts(built, parties, mode, target):
    name, w = target
    M, K, N = 3, 4, 5
    for party in (0, parties // 2, parties - 1):
        L = O.OracleLayer(M, K, N, seed=7, layer_id=4, key_seed=3, parties=parties).deal()
        L[name][party].reshape(-1, 2)[5, 0] ^= np.uint64(1 << 17)
        L.online(mode).check(mode)
        assert L.cs_sums()[w] != 0 and not L.accept(), (name, party)


@pytest.mark.parametrize("parties", [3, 4])
def test_parties_with_truncation_conv_and_compression_along_m(built, parties):
    """n parties with f > 0 (only party 0 subtracts the public term), a
    convolution, and the compression along M."""
    L = O.run_layer(O.MODE_COMPACT, 4, 18, 25, 5, 6, 7, f=9, parties=parties, compress=1,
                    conv=(2, 5, 5, 3, 1, 1))
    assert L.accept()
    dn = sum(int(v) for v in L.delta)
    assert (nlift(L, "tZf") == (dn * nlift(L, "Zf")) % R).all()
    D = ints(L["D"]) % (1 << 64)
    # R^f = (R mod 2^k) / 2^f below 2^k, and the truncated output reconstructs to R^f - (D mod 2^k) / 2^f
    assert (nlift(L, "Rf") % (1 << 64) == (nlift(L, "R") % (1 << 64)) // 2 ** 9).all()
    assert (nlift(L, "Zf") == (nlift(L, "Rf") - D // 2 ** 9) % R).all()
