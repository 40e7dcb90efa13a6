"""Brute-force Wick contractions of dense quark lines for the hadron-correlator pins: the
quark line Q = S Omega^-1 S as a dense matrix over (t, x, spin, colour), written out over
sites, colours and spins with no LapH factorisation (test helper, not part of the oracle
or the product)."""
import itertools

import numpy as np

EPS = np.zeros((3, 3, 3))
for (a, b, c), s in zip(itertools.permutations(range(3)), (1, -1, -1, 1, 1, -1)):
    EPS[a, b, c] = s  # itertools order: 012 021 102 120 201 210


def baryon_wick(Q, ns, nt, t0, c, cp, k):
    """Sec. III.A's six-term Wick contraction for three quark lines of one flavour: for
    every sink slice tF, sum c_abg conj(c'_a'b'g') eps eps e^{-ip.(x - x0)} over the six
    pairings of Q(x tF, x0 t0) (the spin tensors' nonzero entries only)."""
    V3 = ns ** 3
    Qr = Q.reshape(nt, V3, 4, 3, nt, V3, 4, 3)
    cz = np.arange(V3)
    coord = np.stack([cz % ns, (cz // ns) % ns, cz // ns ** 2], axis=1)
    ph = np.exp(-2j * np.pi * coord @ np.array(k) / ns)
    ref = np.zeros(nt, dtype=np.complex128)
    nzc = list(zip(*np.nonzero(c)))
    nzp = list(zip(*np.nonzero(cp)))
    for tf in range(nt):
        q = Qr[tf, :, :, :, t0]  # [x, spin, colour, x0, spin0, colour0]
        tot = 0
        for (al, be, ga) in nzc:
            for (a0, b0, g0) in nzp:
                w = c[al, be, ga] * np.conj(cp[a0, b0, g0])

                def L(s, s0):
                    return q[:, s, :, :, s0, :]

                terms = [(+1, L(al, a0), L(be, b0), L(ga, g0), "xau,xbv,xcw"),
                         (-1, L(al, a0), L(be, g0), L(ga, b0), "xau,xbw,xcv"),
                         (-1, L(al, b0), L(be, a0), L(ga, g0), "xav,xbu,xcw"),
                         (-1, L(al, g0), L(be, b0), L(ga, a0), "xaw,xbv,xcu"),
                         (+1, L(al, g0), L(be, a0), L(ga, b0), "xaw,xbu,xcv"),
                         (+1, L(al, b0), L(be, g0), L(ga, a0), "xav,xbw,xcu")]
                for sign, A1, A2, A3, spec in terms:
                    s1, s2, s3 = spec.split(",")
                    expr = "abc,uvw,x,y,{0},{1},{2}->".format(*[s[0] + s[1] + "y" + s[2] for s in (s1, s2, s3)])
                    tot += sign * w * np.einsum(expr, EPS, EPS, ph, ph.conj(), A1, A2, A3)
        ref[tf] = tot
    return ref
