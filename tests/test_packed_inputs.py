"""The symmetry-packed (tt|cc) / (tc|tc) input layout on the CPU: the packed
generator draws arrays with every symmetry of the two-electron integrals
((pq|jj') symmetric in p, q and in j, j'; (pj|qj') symmetric under
(p, j) <-> (q, j'); zero exactly where the irreps forbid a value, non-zero
elsewhere), packing and unpacking are inverse, and the oracle reads the
packed layout to the same matrix, bit for bit, as the dense arrays."""
import numpy as np

import oracle
import synth


def test_packed_generator_symmetries():
    inst = synth.make_instance(7, 4, 4, [3, 2, 4, 1], [0, 1, 2, 3], 6, 2, 10, 77, packed=True)
    d = synth.unpack_integrals(inst)
    ci, ti = d.cont_irrep.astype(int), d.tgt_irrep.astype(int)
    T, K = d.ttcc, d.tctc
    assert np.array_equal(T, T.transpose(1, 0, 2, 3)) and np.array_equal(T, T.transpose(0, 1, 3, 2))
    assert np.array_equal(K, K.transpose(2, 3, 0, 1))
    mt = (ti[:, None, None, None] ^ ti[None, :, None, None] ^ ci[None, None, :, None] ^ ci[None, None, None, :]) != 0
    mk = (ti[:, None, None, None] ^ ci[None, :, None, None] ^ ti[None, None, :, None] ^ ci[None, None, None, :]) != 0
    assert np.all(T[mt] == 0) and np.all(K[mk] == 0)
    assert np.all(T[~mt] != 0) and np.all(K[~mk] != 0)
    again = synth.pack_integrals(d)
    assert np.array_equal(again.ttcc, inst.ttcc) and np.array_equal(again.tctc, inst.tctc)
    rec, _ = synth.packed_layout(inst.tgt_irrep, inst.n_c)
    assert inst.ttcc.size == rec[-1] == np.count_nonzero(~mt)


def test_oracle_packed_equals_dense():
    dense = synth.make_instance(8, 4, 4, [5, 3, 0, 2], [0, 1, 2, 3], 12, 3, 30, 78)
    packed = synth.pack_integrals(dense)
    H1, A1, K1 = oracle.Oracle(dense).build(with_abs=True)
    H2, A2, K2 = oracle.Oracle(packed).build(with_abs=True)
    assert np.array_equal(H1, H2) and np.array_equal(A1, A2) and np.array_equal(K1, K2)
    assert np.abs(H1[:dense.n_cont_rows(), :dense.n_cont_rows()]).max() > 0
