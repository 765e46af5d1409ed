"""Pins of the randomized-projection oracle (Section 8's 'Rand. Proj.':
eq. (pkLong) with a fresh standard normal sketch each iteration):

* Philox4x32-10 against its published known-answer values;
* Box-Muller against closed forms;
* the sketch's first two moments and the independence of its draws;
* every update is brute-force eq. (pkLong) with the same sketch, satisfies
  the sketched constraints (eq. cons), and the error to A†b never grows
  (each update is an orthogonal projection of it);
* a square sketch (r = m) solves the system in one step."""
import math
import os

import numpy as np

import plss_inputs as gen
from oracle import pins
from oracle import randproj as R

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.txt")


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def test_philox_known_answers():
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        c, k, o = (part.split() for part in line.split(";"))
        got = R.philox4x32_10(np.array([[int(v, 16) for v in c]], dtype=np.uint64),
                              tuple(int(v, 16) for v in k))[0]
        assert [int(v) for v in got] == [int(v, 16) for v in o]


def test_box_muller_closed_forms():
    z0, z1 = R.box_muller(np.array([math.exp(-0.5)]), np.array([0.0]))
    assert abs(z0[0] - 1.0) < 1e-15 and abs(z1[0]) < 1e-15
    z0, z1 = R.box_muller(np.array([math.exp(-2.0)]), np.array([0.25]))
    assert abs(z0[0]) < 1e-15 and abs(z1[0] - 2.0) < 1e-15
    assert R.uniforms([0])[0] == 0.5 * 2.0 ** -32 and R.uniforms([2 ** 32 - 1])[0] < 1.0


def test_sketch_moments_and_independence():
    S = R.sketch(20000, 10, 3, 761511)
    assert abs(S.mean()) < 0.01 and abs(S.std() - 1.0) < 0.01
    assert abs(np.mean(S[:, 0] * S[:, 1])) < 0.03
    # counters differ by iteration and seed; the first r columns of a wider draw agree
    assert not np.allclose(R.sketch(50, 4, 1, 7), R.sketch(50, 4, 2, 7))
    assert not np.allclose(R.sketch(50, 4, 1, 7), R.sketch(50, 4, 1, 8))
    np.testing.assert_array_equal(R.sketch(50, 6, 1, 7), R.sketch(50, 8, 1, 7)[:, :6])


def test_updates_are_bruteforce_pklong():
    sysm = gen.tiny(401, 40, 70, 8)
    D = sysm.A.dense()
    res = R.randproj(sysm.A, sysm.b, r=5, seed=11, tol=1e-300, maxit=12, record=True)
    xm = pins.min_norm(D, sysm.b)
    err = [np.linalg.norm(x - xm) for x in res.xs]
    for k in range(1, 13):
        S = R.sketch(40, 5, k, 11)
        assert rel(res.ps[k - 1], pins.pk_bruteforce(D, S, res.rs[k - 1])) <= 1e-10
        # eq. (cons): S_kᵀ A x_k = S_kᵀ b
        assert np.linalg.norm(S.T @ (sysm.b - D @ res.xs[k])) <= 1e-10 * np.linalg.norm(S.T @ sysm.b)
        assert err[k] <= err[k - 1] * (1 + 1e-12)


def test_square_sketch_solves_in_one_step():
    sysm = gen.tiny(403, 12, 30, 6)
    res = R.randproj(sysm.A, sysm.b, r=12, seed=5, tol=1e-300, maxit=1)
    assert rel(res.x, pins.min_norm(sysm.A.dense(), sysm.b)) <= 1e-10


def test_converges_on_a_small_system():
    sysm = gen.small(m=400, n=100)
    res = R.randproj(sysm.A, sysm.b, r=10, seed=3, tol=1e-6, maxit=5000)
    assert res.status == 0 and res.relres_true <= 1.5e-6
