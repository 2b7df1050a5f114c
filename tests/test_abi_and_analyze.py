"""Host-side tests of the library: ABI exports, ordering validity and the
symbolic analysis, bit-exact against the CPU oracle (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_2007_01541_amd import Symbolic
from paper_2007_01541_amd import capi
from workloads import tiny, small_fp64, WaveletSpec, make_matrix

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"\b(wcs_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = capi.lib()
    names = declared_functions()
    assert len(names) >= 15
    for nm in names:
        assert hasattr(lib, nm), nm
    # and the binding declares each of them
    bound = {s[0] for s in capi.SIGNATURES}
    assert set(names) <= bound, set(names) - bound


def fundamental_partition(parent, colcount):
    """Fundamental supernodes from the definition: j+1 continues j's supernode
    iff parent[j] = j+1, j is j+1's only child, colcount[j] = colcount[j+1] + 1."""
    n = parent.size
    nchild = np.bincount(parent[parent >= 0], minlength=n)
    starts = [0]
    for j in range(1, n):
        if not (parent[j - 1] == j and nchild[j] == 1 and colcount[j - 1] == colcount[j] + 1):
            starts.append(j)
    return np.array(starts + [n], np.int32)


def check_against_oracle(m, sym):
    n = m["n"]
    ex = sym.export()
    inf = sym.info
    assert oracle.check_perm(ex["perm"])
    assert oracle.check_nd(n, m["colptr"], m["rowind"], ex["perm"], ex["sep_tree"]) == 0
    parent, cc, nnzL, flops = oracle.symbolic(n, m["colptr"], m["rowind"], ex["perm"])
    assert np.array_equal(ex["parent"], parent)
    assert np.array_equal(ex["colcount"], cc)
    assert inf["nnz_l"] == nnzL and inf["flops"] == flops
    assert np.array_equal(ex["super_ptr"], fundamental_partition(parent, cc))
    # amalgamated fronts are unions of consecutive fundamental supernodes
    assert set(ex["relaxed_ptr"].tolist()) <= set(ex["super_ptr"].tolist())
    assert inf["flops_padded"] >= inf["flops"]
    return ex


@pytest.mark.parametrize("coords", [True, False])
def test_analyze_small_config_bit_exact(small_matrix, coords):
    m = small_matrix
    sym = Symbolic(m["n"], m["colptr"], m["rowind"], coords=m["coords"] if coords else None)
    check_against_oracle(m, sym)


@pytest.mark.parametrize("G,a,leaf", [(3, 1.2, 4), (4, 1.5, 8), (5, 1.3, 16), (5, 2.0, 64)])
def test_analyze_tiny_bit_exact(G, a, leaf):
    m = tiny(G, a).matrix()
    for coords in (m["coords"], None):
        sym = Symbolic(m["n"], m["colptr"], m["rowind"], coords=coords, leaf_size=leaf, dense_degree_min=16)
        check_against_oracle(m, sym)


def test_analyze_user_perm_and_no_relax():
    m = tiny(4, 1.5).matrix()
    n = m["n"]
    for perm in (np.arange(n, dtype=np.int32), np.random.default_rng(1).permutation(n).astype(np.int32)):
        sym = Symbolic(n, m["colptr"], m["rowind"], user_perm=perm, relax=False)
        ex = check_against_oracle(m, sym)
        assert np.array_equal(ex["perm"], perm)
        assert np.array_equal(ex["relaxed_ptr"], ex["super_ptr"])


def test_analyze_deterministic(small_matrix):
    m = small_matrix
    a = Symbolic(m["n"], m["colptr"], m["rowind"], coords=m["coords"]).export()
    b = Symbolic(m["n"], m["colptr"], m["rowind"], coords=m["coords"]).export()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_nd_reduces_fill_versus_levelwise(small_matrix):
    """Section 4: the levelwise order fills in massively, nested dissection does not."""
    m = small_matrix
    n = m["n"]
    nd = Symbolic(n, m["colptr"], m["rowind"], coords=m["coords"]).info
    nat = Symbolic(n, m["colptr"], m["rowind"], user_perm=np.arange(n, dtype=np.int32)).info
    assert nat["nnz_l"] == n * (n + 1) // 2     # dense
    assert nd["nnz_l"] < nat["nnz_l"] / 4


def _malformed_cases():
    m = tiny(3, 1.5).matrix()
    cp, ri = m["colptr"].copy(), m["rowind"].copy()
    yield "diag missing", cp, np.where(np.arange(ri.size) == cp[3], ri + 1, ri).astype(np.int32)
    r2 = ri.copy(); r2[cp[2] + 1], r2[cp[2] + 2] = r2[cp[2] + 2], r2[cp[2] + 1]
    yield "unsorted", cp, r2
    r3 = ri.copy(); r3[cp[5] + 1] = 10_000
    yield "out of range", cp, r3
    c4 = cp.copy(); c4[0] = 1
    yield "colptr[0]", c4, ri


@pytest.mark.parametrize("case", list(range(4)))
def test_malformed_pattern_is_rejected(case):
    name, cp, ri = list(_malformed_cases())[case]
    with pytest.raises(capi.WcsError) as e:
        Symbolic(cp.size - 1, cp, ri)
    assert e.value.code == -1, name
    assert capi.lib().wcs_last_error().decode()


def test_bad_user_perm_rejected():
    m = tiny(3, 1.5).matrix()
    with pytest.raises(capi.WcsError):
        Symbolic(m["n"], m["colptr"], m["rowind"], user_perm=np.zeros(m["n"], np.int32))


def test_workspace_too_small_is_enomem():
    m = tiny(3, 1.5).matrix()
    sym = Symbolic(m["n"], m["colptr"], m["rowind"], coords=m["coords"])
    need = sym.workspace_size(0, 1)
    h = C.c_void_p()
    fake = 1 << 20       # aligned, never dereferenced: the size check fails first
    rc = capi.lib().wcs_factor_create(sym.handle, 0, 1, fake, need - 1, None, C.byref(h))
    assert rc == -2 and not h.value
    rc = capi.lib().wcs_factor_create(sym.handle, 0, 0, fake, need, None, C.byref(h))
    assert rc == -1


def test_anz_rounding_convention():
    """The paper's anz = nnz/N is printed rounded up (golden values from its tables and figures)."""
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "anz_rounding.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) >= 3
    for nnz, n, printed in rows:
        assert -(-int(nnz) // int(n)) == int(printed)
