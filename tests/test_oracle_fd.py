"""Pins of the oracle's nonzero structure constants (Eq. (11), Table 1 step 2.2)."""
import itertools
import os

import numpy as np
import pytest

import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "su3_gellmann_structure_constants.txt")


def _as_dict(mns, val):
    return {tuple(t): v for t, v in zip(mns.tolist(), val.tolist())}


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_fd_equals_brute_force_traces(oracle, N):
    f, d = brute.structure_constants(N)
    assert np.abs(f.imag).max() < 1e-14 and np.abs(d.imag).max() < 1e-14
    for which, ref in (("f", f.real), ("d", d.real)):
        got = _as_dict(*oracle.fd_enumerate(N, which))
        want = {tuple(t): ref[tuple(t)] for t in np.argwhere(np.abs(ref) > 1e-9)}
        assert set(got) == set(want)
        assert max([abs(got[k] - want[k]) for k in want] + [0.0]) < 1e-13


def test_su3_textbook_tables(oracle):
    pos = None
    entries = []
    for line in open(GOLDEN):
        line = line.strip()
        if line.startswith("# map"):
            pos = {int(t.split("->")[0][6:]): int(t.split("->")[1]) for t in line[6:].split()}
        if not line or line.startswith("#"):
            continue
        kind, a, b, c, v = line.split()
        val = eval(v.replace("sqrt3", "3**0.5"))
        entries.append((kind, int(a), int(b), int(c), val))
    assert pos is not None and len(pos) == 8
    want = {"f": {}, "d": {}}
    for kind, a, b, c, v in entries:
        for perm in itertools.permutations((a, b, c)):
            sign = 1.0
            if kind == "f":
                # parity of the permutation
                p = list(perm)
                inv = sum(1 for i in range(3) for j in range(i + 1, 3) if [a, b, c].index(p[i]) > [a, b, c].index(p[j]))
                sign = -1.0 if inv % 2 else 1.0
            key = tuple(pos[x] for x in perm)
            want[kind][key] = sign * v * np.sqrt(2.0)
    for which in ("f", "d"):
        got = _as_dict(*oracle.fd_enumerate(3, which))
        assert set(got) == set(want[which])
        for k, v in want[which].items():
            assert abs(got[k] - v) < 1e-14, (which, k, got[k], v)


@pytest.mark.parametrize("N", [3, 4, 6, 9])
def test_fd_symmetries(oracle, N):
    f = _as_dict(*oracle.fd_enumerate(N, "f"))
    d = _as_dict(*oracle.fd_enumerate(N, "d"))
    for (a, b, c), v in f.items():
        assert f[(b, c, a)] == pytest.approx(v, abs=1e-14)
        assert f[(b, a, c)] == pytest.approx(-v, abs=1e-14)
    for (a, b, c), v in d.items():
        assert d[(b, c, a)] == pytest.approx(v, abs=1e-14)
        assert d[(b, a, c)] == pytest.approx(v, abs=1e-14)


@pytest.mark.parametrize("N", list(range(2, 13)))
def test_fd_counts_closed_form(oracle, N):
    # Counting the three index classes (triangles of pairs, pair + its partner +
    # a diagonal generator, three diagonal generators) gives
    # 5N^3 - 9N^2 - 2N + 6 ordered nonzero f and 6N^3 - 10.5N^2 - 3.5N + 1 ordered
    # nonzero d; both agree with brute-force traces for N <= 5 above.
    nf, nd = oracle.fd_count(N)
    assert nf == 5 * N**3 - 9 * N**2 - 2 * N + 6
    assert nd == round(6 * N**3 - 10.5 * N**2 - 3.5 * N + 1)


def test_fd_scaling_is_cubic(oracle):
    # Only O(N^3) of the M^3 coefficients are nonzero (Sec. 4, step 2.2)
    nf, nd = oracle.fd_count(16)
    M = 16 * 16 - 1
    assert nf < 6 * 16**3 and nd < 7 * 16**3 and nf < 5e-3 * M**3
