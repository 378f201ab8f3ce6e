"""Oracle pins from the paper's Example 1 (values printed in the paper)."""
import json
import os

import numpy as np
import scipy.sparse as sp

from conftest import GOLDEN
from oracle import geometry, split

EX = json.load(open(os.path.join(GOLDEN, "example1.json")))
A = np.array(EX["A"], dtype=np.float64)
P = np.array(EX["p"], dtype=np.float64)


def test_example1_matrix_is_symmetric_in_the_sense_of_eq2():
    assert geometry.is_symmetric(sp.csr_matrix(A))
    assert np.array_equal(A, A[::-1, ::-1])


def test_example1_fold_reproduces_printed_systems_exactly():
    S = split.fold(sp.csr_matrix(A))
    assert np.array_equal(S.A1().toarray(), np.array(EX["A1"], float))
    assert np.array_equal(S.A2().toarray(), np.array(EX["A2"], float))
    p1, p2 = split.fold_p(P)
    assert np.array_equal(p1, EX["p1"])
    assert np.array_equal(p2, EX["p2"])
    # fp32 fold of small integers is exact too
    S32 = split.fold(sp.csr_matrix(A.astype(np.float32)), "fp32")
    assert np.array_equal(S32.A1().toarray(), np.array(EX["A1"], np.float32))


def test_example1_general_solutions_solve_the_split_and_full_systems():
    A1 = np.array(EX["A1"], float)
    A2 = np.array(EX["A2"], float)
    g1, g2, gf = EX["general_f1"], EX["general_f2"], EX["general_f"]
    for x, y in [(0.0, 0.0), (1.0, -2.0), (0.37, 5.5), (-3.0, 0.125)]:
        f1 = np.array(g1["u"]) * x + np.array(g1["w"])
        f2 = np.array(g2["u"]) * y + np.array(g2["w"])
        assert np.allclose(A1 @ f1, EX["p1"], atol=1e-12)
        assert np.allclose(A2 @ f2, EX["p2"], atol=1e-12)
        # Theorem 1: the recombination solves (12), and equals the printed family
        f = split.recombine(f1, f2)
        assert np.allclose(A @ f, P, atol=1e-12)
        fam = np.array(gf["ux"]) * x + np.array(gf["uy"]) * y + np.array(gf["w"])
        assert np.allclose(f, fam, atol=1e-12)


def test_example1_normal_pseudo_solutions_match_printed_values():
    tol = 0.5 * 10.0 ** -EX["decimals"] + 1e-12
    A1 = np.array(EX["A1"], float)
    A2 = np.array(EX["A2"], float)
    f1 = np.linalg.pinv(A1) @ np.array(EX["p1"], float)
    f2 = np.linalg.pinv(A2) @ np.array(EX["p2"], float)
    assert np.allclose(f1, EX["pseudo_f1"], atol=tol, rtol=0)
    assert np.allclose(f2, EX["pseudo_f2"], atol=tol, rtol=0)
    assert abs(np.linalg.norm(f1) - EX["norm_f1"]) <= tol
    assert abs(np.linalg.norm(f2) - EX["norm_f2"]) <= tol
    # Theorem 2: the recombined halves are the normal pseudo-solution of (12)
    f = split.recombine(f1, f2)
    assert np.allclose(f, EX["pseudo_f"], atol=tol, rtol=0)
    assert abs(np.linalg.norm(f) - EX["norm_f"]) <= tol
    assert np.allclose(f, np.linalg.pinv(A) @ P, atol=1e-13)


def _example1_fold_pin_holds(A1, A2) -> bool:
    return (np.array_equal(A1, np.array(EX["A1"], float))
            and np.array_equal(A2, np.array(EX["A2"], float)))


def test_example1_pin_catches_plausible_fold_mistakes():
    S = split.fold(sp.csr_matrix(A))
    assert _example1_fold_pin_holds(S.A1().toarray(), S.A2().toarray())
    m, n = 2, 3
    top = A[:m, :n]
    mistakes = {
        "sign flipped": (A[::-1][:m, :n] - top, top + A[::-1][:m, :n]),
        # 1-based row i paired with row M-i instead of M-i+1
        "off-by-one row pairing": (top - A[[2, 1], :n], top + A[[2, 1], :n]),
        "mirror row not reversed in columns": (top - A[::-1, ::-1][:m, :n],
                                               top + A[::-1, ::-1][:m, :n]),
        "halves swapped": (top + A[::-1][:m, :n], top - A[::-1][:m, :n]),
    }
    for name, (a1, a2) in mistakes.items():
        assert not _example1_fold_pin_holds(a1, a2), name
