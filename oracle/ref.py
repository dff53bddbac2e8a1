"""Pure-Python big-integer brute force of the same two-party procedure, for tiny
shapes only (test infrastructure).

It is a second, independent transcription of the paper's steps with Python
integers reduced mod 2^128 by hand, used to cross-check the C oracle on inputs
small enough for Python loops.  It reads the C oracle's arrays only as inputs
(the dealt shares) and recomputes every online and verification output.
"""
from __future__ import annotations

MASK64 = (1 << 64) - 1
R128 = 1 << 128
GAMMA = 0x9E3779B97F4A7C15


def mix64(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def draw(seed: int, stream: int, i: int) -> int:
    key = mix64(seed ^ mix64(stream))
    return mix64(key + (i + 1) * GAMMA)


def stream(layer_id: int, purpose: int) -> int:
    return ((layer_id << 16) | purpose) & MASK64


def mat(M, K, N, P, Q, ring=R128):
    return [[sum(P[i][k] * Q[k][j] for k in range(K)) % ring for j in range(N)] for i in range(M)]


def online_and_check(compact: bool, M, K, N, seed, layer_id, delta, S, f: int = 0, kbits: int = 64):
    """S: dict name -> per-party lists of Python-int matrices (X, tX, A, tA, Y, tY,
    B, tB, C, tC, R, tR, and Rf, tRf when f > 0), each S[name][p][i][j].
    Arithmetic is mod 2^{k+s} with k = s = kbits; combiners are draws mod 2^s.
    Returns a dict of outputs."""
    R128 = 1 << (2 * kbits)          # the ring Z_{2^{k+s}} (name kept from the default k = 64)
    smask = (1 << kbits) - 1

    def mat(M_, K_, N_, P, Q):
        return [[sum(P[i][k] * Q[k][j] for k in range(K_)) % R128 for j in range(N_)] for i in range(M_)]
    out = {}
    E = [[(S["X"][0][i][k] - S["A"][0][i][k] + S["X"][1][i][k] - S["A"][1][i][k]) % R128
          for k in range(K)] for i in range(M)]
    U = [[(S["Y"][0][k][j] - S["B"][0][k][j] + S["Y"][1][k][j] - S["B"][1][k][j]) % R128
          for j in range(N)] for k in range(K)]
    EU = mat(M, K, N, E, U)
    Z = []
    for p in range(2):
        EB = mat(M, K, N, E, S["B"][p])
        AU = mat(M, K, N, S["A"][p], U)
        Z.append([[(S["C"][p][i][j] + EB[i][j] + AU[i][j] + (EU[i][j] if p == 0 else 0)) % R128
                   for j in range(N)] for i in range(M)])
    D = [[(S["R"][0][i][j] - Z[0][i][j] + S["R"][1][i][j] - Z[1][i][j]) % R128 for j in range(N)]
         for i in range(M)]
    if f > 0:
        # truncation by the opened D: its value mod 2^64, shifted right by f
        Df = [[(D[i][j] & smask) >> f for j in range(N)] for i in range(M)]
        out["Zf"] = [[[(S["Rf"][p][i][j] - (Df[i][j] if p == 0 else 0)) % R128 for j in range(N)]
                      for i in range(M)] for p in range(2)]
        out["tZf"] = [[[(S["tRf"][p][i][j] - delta[p] * Df[i][j]) % R128 for j in range(N)]
                       for i in range(M)] for p in range(2)]
    tZ = []
    if not compact:
        for p in range(2):
            EtB = mat(M, K, N, E, S["tB"][p])
            tAU = mat(M, K, N, S["tA"][p], U)
            tZ.append([[(S["tC"][p][i][j] + EtB[i][j] + tAU[i][j] + delta[p] * EU[i][j]) % R128
                        for j in range(N)] for i in range(M)])
    else:
        for p in range(2):
            tZ.append([[(S["tR"][p][i][j] - delta[p] * D[i][j]) % R128 for j in range(N)] for i in range(M)])
        chi = [draw(seed, stream(layer_id, 0x30), j) & smask for j in range(N)]
        comp = lambda Mx, rows: [sum(Mx[i][j] * chi[j] for j in range(N)) % R128 for i in range(rows)]
        Uc = comp(U, K)
        Dc = comp(D, M)
        EUc = [sum(E[i][k] * Uc[k] for k in range(K)) % R128 for i in range(M)]
        tZc, tDc = [], []
        for p in range(2):
            tBc = comp(S["tB"][p], K)
            tCc = comp(S["tC"][p], M)
            tRc = comp(S["tR"][p], M)
            z = [(tCc[i] + sum(E[i][k] * tBc[k] for k in range(K)) + sum(S["tA"][p][i][k] * Uc[k] for k in range(K))
                  + delta[p] * EUc[i]) % R128 for i in range(M)]
            tZc.append(z)
            tDc.append([(tRc[i] - z[i]) % R128 for i in range(M)])
        out.update(Uc=Uc, Dc=Dc, EUc=EUc, tZc=tZc, tDc=tDc)
    out.update(E=E, U=U, Z=Z, D=D, tZ=tZ)

    def batch_cs(W, tWp, rows, cols, purpose, p):
        cs = 0
        for i in range(rows):
            for j in range(cols):
                c = draw(seed, stream(layer_id, purpose), i * cols + j) & smask
                cs += tWp[i][j] * c - delta[p] * (W[i][j] * c)
        return cs % R128

    cs = [[0, 0], [0, 0], [0, 0]]
    for p in range(2):
        tE = [[S["tX"][p][i][k] - S["tA"][p][i][k] for k in range(K)] for i in range(M)]
        tU = [[S["tY"][p][k][j] - S["tB"][p][k][j] for j in range(N)] for k in range(K)]
        cs[0][p] = batch_cs(E, tE, M, K, 0x32, p)
        cs[1][p] = batch_cs(U, tU, K, N, 0x33, p)
        if not compact:
            tD = [[S["tR"][p][i][j] - tZ[p][i][j] for j in range(N)] for i in range(M)]
            cs[2][p] = batch_cs(D, tD, M, N, 0x34, p)
        else:
            s = 0
            for i in range(M):
                ch = draw(seed, stream(layer_id, 0x31), i) & smask
                s += (delta[p] * out["Dc"][i]) * ch - out["tDc"][p][i] * ch
            cs[2][p] = s % R128
    out["cs"] = cs
    return out
