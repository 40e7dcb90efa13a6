"""Pins of the oracle's Z4 noise and dilution projectors (CPU only).

Noise: Sec. II (noise vectors in the LapH subspace with E(rho) = 0, E(rho rho^dag) = 1,
Z_N entries giving zero variance on the diagonal) and Sec. IV (Z4 noise named by a
16-bit noise id and a 16-bit configuration id).  The generator is Philox4x32-10, pinned
by its published known-answer vectors and by rocRAND's independent implementation.
Dilution: Sec. II (the four projector families, the (T,S,L) triplet, N/J integral) and
the inversion counts of Sec. II (dilution-scheme discussion).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    rows = []
    with open(os.path.join(GOLD, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(w, 16) for w in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = oracle.philox4x32_10(r[0:4], r[4:6])
        assert list(out) == r[6:10]


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand(tmp_path):
    exe = tmp_path / "dump"
    subprocess.check_call(["hipcc", "-O1", "-o", str(exe), os.path.join(GOLD, "rocrand_philox_dump.cpp")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    s, k = 7, 1234
    m = (k << 16) | s
    nt, nv = 3, 17
    out = subprocess.check_output([str(exe), str(m), str(nt), str(nv)]).decode().split("\n")
    ref = {}
    for line in out:
        if line.strip():
            t, a, n, w = map(int, line.split())
            ref[(t, a, n)] = w
    rho = oracle.z4_noise(s, k, nt, nv)
    z4 = np.array([1, 1j, -1, -1j])
    for (t, a, n), w in ref.items():
        assert oracle.philox4x32_10([n, a, t, 0], [m, 0x4C415048])[0] == w
        assert rho[t, a, n] == z4[w & 3]


def test_z4_values_exact_and_uniform():
    rho = oracle.z4_noise(3, 11, 32, 96)
    # every entry is exactly one of {1, i, -1, -i}: |rho|^2 = 1 with zero variance
    assert np.all((rho.real ** 2 + rho.imag ** 2) == 1.0)
    assert np.all((rho.real == 0) | (rho.imag == 0))
    codes = np.round(np.angle(rho) / (np.pi / 2)).astype(int) % 4
    counts = np.bincount(codes.ravel(), minlength=4)
    n = rho.size
    chi2 = ((counts - n / 4) ** 2 / (n / 4)).sum()
    assert chi2 < 16.27  # 3 dof, p = 0.001


def test_noise_moments_over_noises():
    """E(rho) = 0 and E(rho rho^dag) = 1 estimated over N noises: the diagonal is exactly 1
    for every single noise, off-diagonal elements scatter with std 1/sqrt(N)."""
    nt, nv, N = 2, 8, 400
    R = np.stack([oracle.z4_noise(s, 5, nt, nv).ravel() for s in range(N)])
    mean = R.mean(axis=0)
    assert np.abs(mean).max() < 5.0 / np.sqrt(N)
    C = np.einsum("ri,rj->ij", R, R.conj()) / N
    assert np.all(np.diag(C) == 1.0)
    off = C[~np.eye(C.shape[0], dtype=bool)]
    assert abs(np.sqrt(np.mean(np.abs(off) ** 2)) - 1 / np.sqrt(N)) < 0.2 / np.sqrt(N)


def test_noise_depends_on_both_ids():
    a = oracle.z4_noise(0, 1, 4, 8)
    assert not np.array_equal(a, oracle.z4_noise(1, 1, 4, 8))
    assert not np.array_equal(a, oracle.z4_noise(0, 2, 4, 8))
    # counter-based: elements do not depend on the array extent
    b = oracle.z4_noise(0, 1, 6, 12)
    assert np.array_equal(a, b[:4, :, :8])


def test_parse_dilution():
    assert oracle.parse_dilution("(TF, SF, LI8)", 128, 112) == [1, 0, 1, 0, 3, 8]
    assert oracle.parse_dilution("TI16,SF,LI8", 128, 112) == [3, 16, 1, 0, 3, 8]
    assert oracle.parse_dilution("T1,S1,LB4", 8, 8) == [0, 0, 0, 0, 2, 4]
    with pytest.raises(ValueError):
        oracle.parse_dilution("TI3,SF,LF", 8, 8)      # 8/3 not integral
    with pytest.raises(ValueError):
        oracle.parse_dilution("TF,SB3,LF", 8, 8)      # 4/3 not integral
    with pytest.raises(ValueError):
        oracle.parse_dilution("SF,TF,LF", 8, 8)


@pytest.mark.parametrize("spec", ["TF,SF,LF", "TI4,SB2,LI4", "T1,S1,L1", "TB2,SI2,LB8", "TI8,SF,LB2"])
def test_projector_algebra(spec):
    nt, nv = 8, 8
    sch = oracle.parse_dilution(spec, nt, nv)
    nb = oracle.dilution_count(sch, nt, nv)
    Ps = [oracle.dilution_projector(sch, nt, nv, b) for b in range(nb)]
    # complete set: sum_b P_b = 1, and P_b P_b' = delta_bb' P_b (disjoint 0/1 diagonals)
    assert np.array_equal(sum(Ps), np.ones((nt, 4, nv)))
    for P in Ps:
        assert set(np.unique(P)) <= {0.0, 1.0}
    # exact zeros: R = sum_b P_b rho rho^dag P_b is 1 on the diagonal, 0 across blocks
    rho = oracle.z4_noise(0, 1, nt, nv).ravel()
    R = sum(np.outer(P.ravel() * rho, (P.ravel() * rho).conj()) for P in Ps)
    assert np.all(np.diag(R) == 1.0)
    lab = np.zeros(nt * 4 * nv, dtype=int)
    for b, P in enumerate(Ps):
        lab[P.ravel() > 0] = b
    assert np.all(R[lab[:, None] != lab[None, :]] == 0)


def test_block_interlace_membership():
    # block-J: b = floor(J i / N); interlace-J: b = i mod J (N = 12, J = 4)
    sch_b = [0, 0, 0, 0, 2, 4]
    sch_i = [0, 0, 0, 0, 3, 4]
    for b in range(4):
        Pb = oracle.dilution_projector(sch_b, 1, 12, b)[0, 0]
        Pi = oracle.dilution_projector(sch_i, 1, 12, b)[0, 0]
        assert list(np.nonzero(Pb)[0]) == [3 * b, 3 * b + 1, 3 * b + 2]
        assert list(np.nonzero(Pi)[0]) == [b, b + 4, b + 8]


def test_inversion_counts():
    """Counts quoted in Sec. II: 128 per noise for (TF with 4 source times, SF, LI8), 512
    for (TI16, SF, LI8), 5*128 + 2*512 = 1664 per configuration; exact treatment needs
    N_v N_t N_d = 57,344 (24^3 x 128, N_v = 112) and 270,336 (32^3 x 256, N_v = 264)."""
    tf = oracle.parse_dilution("TF,SF,LI8", 128, 112)
    assert oracle.dilution_count(tf, 128, 112) == 128 * 32
    assert 4 * oracle.dilution_count(tf, 128, 112) // 128 == 128
    ti = oracle.parse_dilution("TI16,SF,LI8", 128, 112)
    assert oracle.dilution_count(ti, 128, 112) == 512
    assert 5 * 128 + 2 * 512 == 1664
    full = oracle.parse_dilution("TF,SF,LF", 128, 112)
    assert oracle.dilution_count(full, 128, 112) == 57344
    assert oracle.dilution_count(oracle.parse_dilution("TF,SF,LF", 256, 264), 256, 264) == 270336
    assert oracle.dilution_count(oracle.parse_dilution("TF,SF,LF", 8, 8), 8, 8) == 256
    assert oracle.dilution_count(oracle.parse_dilution("TI16,SF,LI8", 32, 48), 32, 48) == 512
