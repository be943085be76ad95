"""Pins of the oracle's 3x3 block Jacobi (Algorithm 1, "diag[ ]").

The oracle's ``fem.diag_blocks`` reads the nodal 3x3 diagonal blocks out of
the assembled K, and ``solve.block_jacobi_inverse`` inverts them after
replacing fixed rows and columns by the identity.  Both are checked here
against a brute force built element by element from ``element_stiffness_p2``
(itself pinned by the strain-energy tests): the block of node v is the sum,
over the elements containing v, of the element's own 3x3 diagonal block at
v's local position.  A preconditioner error would not show in converged
solves (CG converges under any SPD preconditioner), hence these direct pins.
"""
import numpy as np

from oracle import fem, solve
from paper_1710_08679_amd import meshgen


def brute_force_blocks(m):
    blocks = np.zeros((m.n_nodes, 3, 3))
    for e in range(m.n_elem):
        Ke = fem.element_stiffness_p2(m.xyz[m.conn[e]][None], m.young[e:e + 1], m.poisson[e:e + 1])[0]
        for a in range(10):
            v = m.conn[e, a]
            for i in range(3):
                for j in range(3):
                    blocks[v, i, j] += Ke[3 * a + i, 3 * a + j]
    return blocks


def roller_mesh():
    m = meshgen.kuhn_mesh(2, 2, 2, jitter=0.2, rng=meshgen.rng_for(91, 0))
    meshgen.set_layers_flat(m)
    fixed = np.zeros((m.n_nodes, 3), np.uint8)
    fixed[meshgen.face_nodes(m, 0, 0), 0] = 1   # roller: only x fixed on x = 0
    fixed[meshgen.face_nodes(m, 2, 0), 2] = 1   # roller: only z fixed on z = 0
    return m, fixed


def test_diag_blocks_equal_element_sums():
    m, _ = roller_mesh()
    K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
    ref = brute_force_blocks(m)
    got = fem.diag_blocks(K, m.n_nodes)
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
    # blocks of an SPD-on-free-DOFs operator: symmetric, positive diagonal
    assert np.abs(got - got.transpose(0, 2, 1)).max() <= 1e-14 * np.abs(ref).max()
    assert np.all(np.diagonal(got, axis1=1, axis2=2) > 0)


def test_single_element_blocks_are_the_element_diagonal():
    m = meshgen.kuhn_mesh(1, 1, 1, jitter=0.0)
    one = np.array(m.conn[:1])
    used = np.unique(one)
    remap = -np.ones(m.n_nodes, np.int64)
    remap[used] = np.arange(used.size)
    conn = remap[one]
    xyz = m.xyz[used]
    K = fem.assemble(xyz, conn, 2.5, 0.3)
    Ke = fem.element_stiffness_p2(xyz[conn[0]][None], np.array([2.5]), np.array([0.3]))[0]
    got = fem.diag_blocks(K, used.size)
    for a in range(10):
        v = conn[0, a]
        assert np.array_equal(got[v], Ke[3 * a:3 * a + 3, 3 * a:3 * a + 3])


def test_block_jacobi_inverse_identity_at_fixed_and_inverse_on_free():
    m, fixed = roller_mesh()
    K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
    B = brute_force_blocks(m)
    Minv = solve.block_jacobi_inverse(K, fixed, m.n_nodes)
    eye = np.eye(3)
    n_partial = 0
    for v in range(m.n_nodes):
        fx = [c for c in range(3) if fixed[v, c]]
        fr = [c for c in range(3) if not fixed[v, c]]
        n_partial += 0 < len(fx) < 3
        for c in fx:   # fixed row and column: identity, whatever the coupling in K
            assert np.array_equal(Minv[v, c, :], eye[c])
            assert np.array_equal(Minv[v, :, c], eye[c])
        if fr:          # free part: the inverse of the free sub-block of the element sums
            sub = B[v][np.ix_(fr, fr)]
            prod = Minv[v][np.ix_(fr, fr)] @ sub
            assert np.abs(prod - np.eye(len(fr))).max() <= 1e-12, (v, prod)
    assert n_partial > 0  # the rollers leave nodes with mixed fixed and free DOFs
    # the nodes on the x = 0 roller have nonzero x-coupling in K, so a version
    # that kept the fixed row's off-diagonal entries could not meet the above
    on = meshgen.face_nodes(m, 0, 0)
    assert np.abs(B[on][:, 0, 1:]).max() > 1e-3 * np.abs(B).max()
