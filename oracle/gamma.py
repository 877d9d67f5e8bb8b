"""Euclidean Dirac matrices (oracle; test infrastructure only).

The paper uses the Wilson-clover operator (Sec. 3.1) without fixing a spinor basis. The
oracle takes the DeGrand-Rossi chiral basis: Hermitian gamma_mu with
{gamma_mu, gamma_nu} = 2 delta_mu,nu and gamma_5 = gamma_x gamma_y gamma_z gamma_t =
diag(1, 1, -1, -1). Any basis with these properties gives the same spectrum; the
choice only has to agree with the GPU library's, which the Clifford and free-field
tests pin on both sides.
"""
import numpy as np

_i = 1j

GAMMA = np.array([
    # gamma_x
    [[0, 0, 0, _i], [0, 0, _i, 0], [0, -_i, 0, 0], [-_i, 0, 0, 0]],
    # gamma_y
    [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],
    # gamma_z
    [[0, 0, _i, 0], [0, 0, 0, -_i], [-_i, 0, 0, 0], [0, _i, 0, 0]],
    # gamma_t
    [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],
], dtype=np.complex128)

GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]

ONE = np.eye(4, dtype=np.complex128)

