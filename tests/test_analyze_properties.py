"""Property-based sweep of the symbolic analysis against the oracle (CPU).

Hypothesis draws instances of the synthetic wavelet pattern over grid sides
2^3 .. 2^5, cut-off a in [1.2, 2], s in {1/4, 1/2, 3/4}, value kind and seed,
and analysis options (leaf size, dense-vertex threshold, coordinates or
graph-only splits, relaxation); for each, the library's analysis must pass
the oracle's nested dissection check and equal its symbolic factorization bit
for bit (Lemma 4.1: the pattern of L is fixed by the ordering)."""
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

from paper_2007_01541_amd import Symbolic
from tests.test_abi_and_analyze import check_against_oracle
from workloads import WaveletSpec, make_matrix


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(G=st.integers(3, 5), a=st.floats(1.2, 2.0), s=st.sampled_from([0.25, 0.5, 0.75]),
       kind=st.sampled_from(["exp", "alg"]), seed=st.integers(0, 2 ** 20), leaf=st.sampled_from([4, 8, 16, 32, 64]),
       dense=st.sampled_from([16, 64, 1024]), coords=st.booleans(), relax=st.booleans())
def test_analysis_matches_oracle_property(G, a, s, kind, seed, leaf, dense, coords, relax):
    m = make_matrix(WaveletSpec(G, a, s, kind, 0.3, 1.5, seed))
    sym = Symbolic(m["n"], m["colptr"], m["rowind"], coords=m["coords"] if coords else None, leaf_size=leaf,
                   dense_degree_min=dense, relax=relax)
    ex = check_against_oracle(m, sym)
    if not relax:
        assert (ex["relaxed_ptr"] == ex["super_ptr"]).all()
