"""UAI-format model, evidence and query files (host code, no GPU).

The files are written here by hand in the competition's text format; what
the library reads back (tn_network_get) must equal the tables written, and
malformed files must fail with TN_E_INVALID naming the problem.  The tree
planner then runs on the loaded model and the oracle's log Z of the loaded
tables equals the brute-force value of the hand-written model.
"""
import math

import numpy as np
import pytest

import oracle
import oracle.brute as bf
from paper_2405_14060_amd import workloads as W

MARKOV = """MARKOV
3
2 2 3
3
1 0
2 0 1
2 1 2
2
 0.436 0.564
4
 0.128 0.872
 0.920 0.080
6
0.210 0.333 0.457
0.811 0.000
0.189
"""

BAYES = """BAYES
3 2 2 3 3
1 0
2 0 1
2 1 2
2 0.3 0.7
4 0.9 0.1 0.2 0.8
6 0.5 0.25 0.25 0.1 0.6 0.3
"""


@pytest.fixture(scope="module")
def T():
    import paper_2405_14060_amd as T
    T.lib()
    return T


def write(tmp_path, name, text):
    p = tmp_path / name
    p.write_text(text)
    return str(p)


def test_markov_file_reads_back(T, tmp_path):
    N = T.Network.from_uai(write(tmp_path, "m.uai", MARKOV))
    src = N.src
    assert N.n_vars == 3 and list(N.card) == [2, 2, 3]
    assert [list(s) for s in src.scopes] == [[0], [0, 1], [1, 2]]
    assert not src.is_log
    assert np.allclose(src.values[0], [0.436, 0.564], rtol=0, atol=0)
    assert np.allclose(src.values[1], [0.128, 0.872, 0.920, 0.080], rtol=0, atol=0)
    assert np.allclose(src.values[2], [0.210, 0.333, 0.457, 0.811, 0.000, 0.189], rtol=0, atol=0)
    # Z by hand: sum_x0 f0(x0) sum_x1 f1(x0, x1) sum_x2 f2(x1, x2)
    f0 = np.array([0.436, 0.564])
    f1 = np.array([[0.128, 0.872], [0.920, 0.080]])
    f2 = np.array([[0.210, 0.333, 0.457], [0.811, 0.000, 0.189]])
    z = float(f0 @ f1 @ f2.sum(axis=1))
    assert abs(bf.log_z(src) - math.log(z)) <= 1e-12
    assert abs(oracle.log_z(src) - math.log(z)) <= 1e-12
    pairs, n_leaves, info = T.plan_tree_host(N)
    assert n_leaves == 3 + 3 and pairs.shape == (n_leaves - 1, 2)


def test_bayes_file_is_normalised(T, tmp_path):
    """CPTs with the child last in each scope: without evidence Z = 1, and
    evidence on the root gives p(e) = CPT_root(e)."""
    N = T.Network.from_uai(write(tmp_path, "b.uai", BAYES))
    src = N.src
    assert abs(bf.log_z(src)) <= 1e-12
    ev = np.array([1, -1, -1], np.int32)
    assert abs(bf.log_z(src, ev) - math.log(0.7)) <= 1e-12


def test_evidence_and_query_files(T, tmp_path):
    N = T.Network.from_uai(write(tmp_path, "m.uai", MARKOV))
    one = N.read_uai_evidence(write(tmp_path, "one.evid", "2 0 1 2 2\n"))
    assert one.tolist() == [[1, -1, 2]]
    none = N.read_uai_evidence(write(tmp_path, "none.evid", "0\n"))
    assert none.tolist() == [[-1, -1, -1]]
    many = N.read_uai_evidence(write(tmp_path, "many.evid", "3\n1 1 0\n0\n2 2 1 0 0\n"))
    assert many.tolist() == [[-1, 0, -1], [-1, -1, -1], [0, -1, 1]]
    q = N.read_uai_query(write(tmp_path, "q.query", "2 2 0\n"))
    assert q.tolist() == [2, 0]


@pytest.mark.parametrize("text,what", [
    ("GRID\n1\n2\n0\n", "preamble"),
    ("MARKOV\n2\n2 2\n1\n2 0 1\n3\n1 2 3\n", "entries"),
    ("MARKOV\n2\n2 2\n1\n2 0 5\n4\n1 2 3 4\n", "out of range"),
    ("MARKOV\n2\n2 2\n1\n2 0 1\n4\n1 2 x 4\n", "not a number"),
    ("MARKOV\n2\n2 2\n1\n2 0 1\n4\n1 2 3\n", "file ends"),
    ("MARKOV\n2\n2 2\n1\n2 0 0\n4\n1 2 3 4\n", ""),
    ("MARKOV\n2\n2 2\n1\n2 0 1\n4\n1 2 3 4 5\n", "unexpected"),
    ("MARKOV\n2\n2 2\n1\n2 0 1\n4\n1 -2 3 4\n", ""),
])
def test_malformed_model_files(T, tmp_path, text, what):
    with pytest.raises(T.TNError) as e:
        T.Network.from_uai(write(tmp_path, "bad.uai", text))
    assert e.value.status == 1  # TN_E_INVALID
    assert what in str(e.value)


@pytest.mark.parametrize("text", ["2 0 1\n", "1 0 5\n", "1 7 0\n", "2 0 1 0 0\n", "", "2\n1 0 1\n"])
def test_malformed_evidence_files(T, tmp_path, text):
    N = T.Network.from_uai(write(tmp_path, "m.uai", MARKOV))
    with pytest.raises(T.TNError):
        N.read_uai_evidence(write(tmp_path, "bad.evid", text))


def test_missing_file(T, tmp_path):
    with pytest.raises(T.TNError) as e:
        T.Network.from_uai(str(tmp_path / "absent.uai"))
    assert "cannot open" in str(e.value)


def test_round_trip_of_a_generated_model(T, tmp_path):
    """A generated Bayesian network written in the format and read back:
    identical tables, same log Z by the oracle."""
    bn = W.random_bn(40, seed=2)
    lines = ["BAYES", str(bn.n_vars), " ".join(str(int(c)) for c in bn.card), str(bn.n_factors)]
    for s in bn.scopes:
        lines.append(" ".join([str(len(s))] + [str(int(v)) for v in s]))
    for v in bn.values:
        lines.append(str(len(v)) + " " + " ".join(repr(float(x)) for x in v))
    N = T.Network.from_uai(write(tmp_path, "bn.uai", "\n".join(lines) + "\n"))
    for a, b in zip(N.src.values, bn.values):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    assert abs(oracle.log_z(N.src) - oracle.log_z(bn)) <= 1e-12
