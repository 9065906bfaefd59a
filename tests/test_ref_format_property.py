"""Property test of the reference format builder: for random small matrices
and random options, the format satisfies its invariants, decodes back to
exactly the input entries and multiplies like the plain definition."""
import numpy as np
from hypothesis import given, settings
from hypothesis import strategies as st

import graphgen as gg
import oracle
from oracle import ref_format as rf
from test_ref_format import check_invariants


@settings(max_examples=40, deadline=None)
@given(n_rows=st.integers(1, 60), n_cols=st.integers(1, 60), density=st.floats(0.0, 0.4),
       seed=st.integers(0, 10 ** 6), W=st.integers(1, 70), wl=st.integers(1, 200),
       S=st.sampled_from([1, 2, 4, 8, 64]), split=st.sampled_from([-1, 0, 3, 10]),
       power=st.sampled_from([None, 0.8, 1.5]), camping=st.booleans())
def test_random_formats(n_rows, n_cols, density, seed, W, wl, S, split, power, camping):
    csr = gg.random_csr(n_rows, n_cols, density, seed, power=power)
    fmt = rf.build(csr, W=W, wl=[wl] * 100, S=S, split_len=split, camping_pad=camping)
    check_invariants(csr, fmt)
    x = gg.uniform_f32(n_cols, seed)
    assert np.allclose(rf.spmv_format(fmt, x), oracle.spmv(csr, x), rtol=1e-12, atol=1e-14)
