"""Index algebra of the matrix-core derivatives of 16-node elements, on the CPU.

The local procedure of 2D elements with N = 3 in FP64 computes its x and y
derivatives with v_mfma_f64_4x4x4 (four 4x4x4 products per wavefront).
The lane layout of that instruction was measured on the chip with one-hot
operands: block b reads A[i][k] from lane 16k + 4b + i and B[k][j] from
lane 16k + 4b + j, and leaves D[i][j] on lane 16i + 4b + j.  The kernels
lay node (p, q) of the wavefront's element b on lane 16q + 4b + p.

This emulates the instruction with that layout and checks the operand
choices the kernels make: one product for the y derivative, a product with
the identity (a transpose) and one more for the x derivative, and the
element sums that pair the nodes as the 16-lane DPP row reduction does.
No GPU is needed; the GPU parity tests check the kernels themselves.
"""
import numpy as np

LANES = 64


def mfma4(a, b, c):
    """v_mfma_f64_4x4x4 on 64-lane vectors a, b, c (the measured layout)."""
    d = np.empty(LANES)
    for blk in range(4):
        A = np.array([[a[16 * k + 4 * blk + i] for k in range(4)] for i in range(4)])
        B = np.array([[b[16 * k + 4 * blk + j] for j in range(4)] for k in range(4)])
        C = np.array([[c[16 * i + 4 * blk + j] for j in range(4)] for i in range(4)])
        D = A @ B + C
        for i in range(4):
            for j in range(4):
                d[16 * i + 4 * blk + j] = D[i, j]
    return d


def lane(b, p, q):
    return 16 * q + 4 * b + p


def scatter(fields):
    """fields[b][p][q] -> lane vector in the kernels' element layout."""
    v = np.empty(LANES)
    for b in range(4):
        for p in range(4):
            for q in range(4):
                v[lane(b, p, q)] = fields[b][p][q]
    return v


def lane_pq():
    p = np.empty(LANES, dtype=int)
    q = np.empty(LANES, dtype=int)
    for b in range(4):
        for pp in range(4):
            for qq in range(4):
                p[lane(b, pp, qq)] = pp
                q[lane(b, pp, qq)] = qq
    return p, q


def test_lane_map_is_a_bijection():
    seen = sorted(lane(b, p, q) for b in range(4) for p in range(4) for q in range(4))
    assert seen == list(range(LANES))


def test_products_give_both_derivatives():
    rng = np.random.default_rng(3)
    D = rng.standard_normal((4, 4))           # a derivative matrix (rows: output node)
    idx, idy = 1.7, 0.6
    f = rng.standard_normal((4, 4, 4))        # per element b: f[b][p][q]
    g = rng.standard_normal((4, 4, 4))
    p, q = lane_pq()
    cAy = D[p, q] * idy                       # the y product's A: D[p][q] on node (p, q)
    cBx = D[p, q] * idx                       # the x product's B: the same entries
    cI = (p == q).astype(float)               # the identity
    ydiv = mfma4(cAy, scatter(g), np.zeros(LANES))
    ft = mfma4(scatter(f), cI, np.zeros(LANES))
    div = mfma4(ft, cBx, ydiv)
    want = np.empty((4, 4, 4))
    for b in range(4):
        want[b] = idx * D @ f[b] + idy * g[b] @ D.T     # d/dx over p, d/dy over q
    np.testing.assert_allclose(div, scatter(want), rtol=1e-13, atol=1e-13)
    # the transpose alone: node (q, p)'s value on node (p, q)'s lane, exactly
    assert np.array_equal(ft, scatter(np.transpose(f, (0, 2, 1))))


def test_a_wrong_operand_is_caught():
    # the x derivative taken from f in place of its transpose gives the
    # contraction over q instead (a mistake the product would make silently)
    rng = np.random.default_rng(4)
    D = rng.standard_normal((4, 4))
    f = rng.standard_normal((4, 4, 4))
    p, q = lane_pq()
    wrong = mfma4(scatter(f), D[p, q], np.zeros(LANES))
    right = scatter(np.stack([D @ f[b] for b in range(4)]))
    assert not np.allclose(wrong, right)


def test_element_sums_pair_nodes_as_the_dpp_row_reduction():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((4, 4, 4)) * 10.0 ** rng.integers(-8, 8, (4, 4, 4))
    # the DPP row reduction on node index k = 4q + p: partners 8, 4, 2, 1 apart
    # (rotations; every lane ends with the same bits)
    row = [[x[b][k % 4][k // 4] for k in range(16)] for b in range(4)]
    dpp = []
    for b in range(4):
        y = list(row[b])
        for s in (8, 4, 2, 1):
            y = [y[k] + y[(k - s) % 16] for k in range(16)]
        assert len(set(y)) == 1
        dpp.append(y[0])
    # the matrix-core layout: lanes 32 apart, 16 apart, quad xor 2, quad xor 1
    v = scatter(x)
    for m in (32, 16, 2, 1):
        v = np.array([v[l] + v[l ^ m] for l in range(LANES)])
    for b in range(4):
        vals = {v[lane(b, pp, qq)] for pp in range(4) for qq in range(4)}
        assert vals == {dpp[b]}
