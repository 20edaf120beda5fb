"""Host-side checks of the HIP library (no GPU needed): it loads, exports
every symbol its header declares, and its host logic (pattern compiler,
random stream, Q16 tables) agrees with the oracle."""

import os
import re
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import judges
from oracle.pattern import compile_pattern
from test_oracle_primitives import _kat

A = pytest.importorskip("paper_2601_01388_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _built():
    if not os.path.exists(A.LIB_PATH):
        from paper_2601_01388_amd import build
        build.build()
    A.lib()


def _header_symbols():
    text = open(os.path.join(ROOT, "include", "agis.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(agis_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    syms = _header_symbols()
    assert len(syms) >= 13
    L = A.lib()
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(A.EXPORTED) == syms


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_library_philox_known_answers(ctr, key, out):
    assert A.agis_philox4x32_10(ctr, key) == out


def test_library_fixed_point_tables_match_oracle():
    lt, et = A.agis_fixed_point_tables()
    olt, oet = oracle.fixed_point_tables()
    assert (lt == olt).all() and (et == oet).all()


def _patterns():
    pats = list(synth.NAMED_PATTERNS.values())
    pats = [p for p in pats if p.k >= 2]
    pats += [p for p, _ in synth.random_pattern_set(32, seed=3)]
    return pats


BETAS = [((4, 5), Fraction(4, 5)), ((5, 6), Fraction(5, 6)), ((1, 2), Fraction(1, 2)), ((1, 1), Fraction(1)),
         ((1, 0), float("inf")), ((-1, 0), float("-inf"))]


@pytest.mark.parametrize("mode", ["uniform", "switch", "always", "learned"])
def test_library_pattern_compiler_matches_oracle(mode):
    for p in _patterns():
        for (bn, bd), bf in (BETAS if mode in ("switch", "learned") else BETAS[:1]):
            ref = compile_pattern(p.k, p.edges, mode=mode, beta=bf)
            got = A.agis_compile_pattern(A.make_pattern(p.k, p.adj8()), params=A.make_params(mode=mode, beta=(bn, bd)))
            assert got.k == p.k and got.aut == ref["aut"]
            assert list(got.order[:p.k]) == ref["order"], p
            for i, s in enumerate(ref["steps"]):
                assert (got.bmask[i], got.b[i], got.f1[i], got.i1[i], got.ie[i], got.f2[i]) == \
                    (s["bmask"], s["b"], s["f1"], s["i1"], s["ie"], s["f2"]), (p, i)
                assert Fraction(got.cert_num[i], got.cert_den[i]) == s["certainty"]
                assert got.decision[i] == s["decision"], (p, i, mode, bf)


def test_library_compiler_with_given_order():
    p = synth.named_pattern("house")
    order = [4, 0, 1, 2, 3]
    ref = compile_pattern(p.k, p.edges, order=order)
    got = A.agis_compile_pattern(A.make_pattern(p.k, p.adj8()), order=order)
    assert list(got.order[:5]) == order
    assert [got.decision[i] for i in range(5)] == [s["decision"] for s in ref["steps"]]


def test_library_compiler_errors():
    bad = A.make_pattern(4, [0b0010, 0b0001, 0b1000, 0b0100])  # two components
    with pytest.raises(A.AgisError) as e:
        A.agis_compile_pattern(bad)
    assert e.value.code == A.AGIS_E_PATTERN
    with pytest.raises(A.AgisError) as e:
        A.agis_compile_pattern(A.make_pattern(9, [0] * 8))
    assert e.value.code == A.AGIS_E_PATTERN
    path = synth.named_pattern("4-path")
    with pytest.raises(A.AgisError) as e:
        A.agis_compile_pattern(A.make_pattern(path.k, path.adj8()), order=[0, 2, 1, 3])
    assert e.value.code == A.AGIS_E_ORDER
    with pytest.raises(A.AgisError) as e:
        A.agis_compile_pattern(A.make_pattern(path.k, path.adj8()), order=[0, 1, 1, 3])
    assert e.value.code == A.AGIS_E_ORDER
    asym = A.make_pattern(3, [0b010, 0b000, 0b000])
    with pytest.raises(A.AgisError) as e:
        A.agis_compile_pattern(asym)
    assert e.value.code == A.AGIS_E_PATTERN


def test_product_path_has_no_oracle_or_cpu_fallback():
    # The library package and its sources never reference the oracle.
    pkg = os.path.join(ROOT, "paper_2601_01388_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower() or f == "__init__.py" and "oracle" not in text, f
                assert "import oracle" not in text and "from oracle" not in text


@pytest.mark.parametrize("k", [4, 5])
def test_library_concentrations_match_oracle(k):
    """agis_concentrations (host code of the library) against the oracle's
    inversion on exact copy counts."""
    from oracle import concentration as conc
    from oracle.pattern import automorphisms
    pats = synth.patterns.connected_patterns(k)
    tup = [(p.k, list(p.edges)) for p in pats]
    g = synth.graphs.tiny_graph(8, 0.5, 77)
    copies = [judges.brute_force(g, p.k, p.edges) // automorphisms(p.k, p.edges) for p in pats]
    ce, ind, ci = A.agis_concentrations([A.make_pattern(p.k, p.adj8()) for p in pats], copies)
    ref = conc.induced_from_copies(tup, copies)
    assert np.allclose(ind, [float(x) for x in ref], rtol=1e-12, atol=1e-9)
    assert np.allclose(ce, [float(x) for x in conc.normalise(copies)], rtol=1e-12)
    assert np.allclose(ci, [float(x) for x in conc.normalise(ref)], rtol=1e-12)


def test_library_concentrations_rejects_incomplete_sets():
    pats = synth.patterns.connected_patterns(4)
    ps = [A.make_pattern(p.k, p.adj8()) for p in pats]
    with pytest.raises(A.AgisError):
        A.agis_concentrations(ps[:-1], [1.0] * 5)  # the 4-clique is missing
    with pytest.raises(A.AgisError):
        A.agis_concentrations(ps + [ps[0]], [1.0] * 7)  # duplicate


def test_library_connected_patterns_are_the_isomorphism_classes():
    """agis_connected_patterns against an independent enumeration (the
    oracle's canonical forms of every connected graph on k vertices)."""
    from oracle import concentration as conc
    import itertools
    for k, count in ((2, 1), (3, 2), (4, 6), (5, 21)):
        got = A.agis_connected_patterns(k)
        assert len(got) == count
        codes = set()
        for p in got:
            edges = [(a, b) for a in range(k) for b in range(a + 1, k) if p.adj[a] >> b & 1]
            codes.add(conc._canon(k, edges))
        ref = set()
        pairs = list(itertools.combinations(range(k), 2))
        for m in range(1 << len(pairs)):
            e = [pairs[j] for j in range(len(pairs)) if m >> j & 1]
            if synth.Pattern(k=k, edges=tuple(e)).is_connected():
                ref.add(conc._canon(k, e))
        assert codes == ref
        sizes = [sum(bin(p.adj[a]).count("1") for a in range(k)) // 2 for p in got]
        assert sizes == sorted(sizes)


def test_sampler_division_multipliers_are_exact():
    # The grouped position search divides by G + 1 (17 or 9) as a multiply-
    # high by m and a right shift by s.  That equals floor(x / d) for every
    # 32-bit x when m = ceil(2^(32+s) / d) and m d - 2^(32+s) <= 2^s
    # (Granlund and Montgomery, PLDI 1994); checked here on the constants
    # the kernel source holds, and on boundary values.
    src = open(os.path.join(ROOT, "paper_2601_01388_amd", "csrc", "kernels.hip")).read()
    mg = re.search(r"const uint32_t mg = nq <= 4 \? (0x[0-9A-Fa-f]+)u : (0x[0-9A-Fa-f]+)u;", src)
    ms = re.search(r"const uint32_t ms = nq <= 4 \? (\d+)u : (\d+)u;", src)
    assert mg and ms
    for d, m, s in [(17, int(mg.group(1), 16), int(ms.group(1))), (9, int(mg.group(2), 16), int(ms.group(2)))]:
        assert m == -(-(1 << (32 + s)) // d) and m * d - (1 << (32 + s)) <= (1 << s)
        for x in [0, 1, d - 1, d, d + 1, (1 << 32) - 1, (1 << 32) - d, (1 << 31) + 5] + list(range(0, 5000)):
            assert ((x * m) >> 32) >> s == x // d


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus N with N > 1 exits with status 2 and
    says so, before touching a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert r.returncode == 2, (r.returncode, r.stderr[-500:])
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
