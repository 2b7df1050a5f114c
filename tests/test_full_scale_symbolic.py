"""Symbolic analysis at the benchmark sizes, bit-exact against the oracle (CPU).

Lemma 4.1 fixes the pattern of L given the ordering, so the elimination tree,
the column counts (their sum is nnz(L)), the flop count and the fundamental
supernode partition computed by the library's analysis must equal the
oracle's, which reaches them by a different route (row subtrees), and the
ordering must satisfy the nested dissection block structure of Section 4.
N = 65,536 runs in the default CPU suite; N = 2^18 (the headline matrix,
about half a minute on one core) is marked slow but still runs there.
"""
import time

import numpy as np
import pytest

import workloads
from paper_2007_01541_amd import Symbolic
from tests.test_abi_and_analyze import check_against_oracle


def _check(w):
    t0 = time.perf_counter()
    m = w.matrix()
    t1 = time.perf_counter()
    sym = Symbolic(m["n"], m["colptr"], m["rowind"], coords=m["coords"])
    t2 = time.perf_counter()
    ex = check_against_oracle(m, sym)
    t3 = time.perf_counter()
    inf = sym.info
    print(f"{w.name}: n={m['n']} nnz(L)={inf['nnz_l']} flops={inf['flops']:.4e} fronts={inf['nsuper']}; "
          f"generate {t1 - t0:.1f}s, analyze {t2 - t1:.1f}s, oracle checks {t3 - t2:.1f}s")
    # the colcounts sum to nnz(L) and their squares to the flop count (R27)
    cc = ex["colcount"].astype(np.int64)
    assert int(cc.sum()) == inf["nnz_l"] and int((cc * cc).sum()) == inf["flops"]
    return m, sym


def test_analyze_n65536_bit_exact():
    _check(workloads.medium_fp64())


@pytest.mark.slow
def test_analyze_headline_n262144_bit_exact():
    m, sym = _check(workloads.headline())
    inf = sym.info
    # the figures every benchmark line quotes for this matrix
    assert inf["n"] == 262144 and inf["nnz_lower"] == 106807042
