"""The seeded synthetic inputs: the gauge links are SU(3) to rounding, so the third row of
every link equals conj(row 1 x row 2), the identity the hop kernels use to store two rows
per link; and the generator is reproducible seed by seed."""
import numpy as np

import synth


def test_gauge_links_are_su3_and_third_row_follows_from_the_first_two():
    U = synth.gauge_field((4, 4, 2, 2), 0.5, 21).reshape(-1, 3, 3)
    eye = np.eye(3)
    assert np.max(np.abs(np.conj(np.swapaxes(U, -1, -2)) @ U - eye)) <= 1e-14
    assert np.max(np.abs(np.linalg.det(U) - 1.0)) <= 1e-14
    row3 = np.conj(np.cross(U[:, 0, :], U[:, 1, :]))
    assert np.max(np.abs(row3 - U[:, 2, :])) <= 1e-14
    # a U(3) link with det != 1 is not recovered: the identity needs unit determinant
    V = U[:5] * np.exp(0.3j)
    assert np.max(np.abs(np.conj(np.cross(V[:, 0, :], V[:, 1, :])) - V[:, 2, :])) > 1e-2


def test_generator_is_reproducible_per_seed():
    a = synth.gauge_field((2, 2, 2, 2), 0.35, 7)
    b = synth.gauge_field((2, 2, 2, 2), 0.35, 7)
    c = synth.gauge_field((2, 2, 2, 2), 0.35, 8)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert np.array_equal(synth.gaussian_spinor((2, 2, 2, 2), 3, nrhs=2),
                          synth.gaussian_spinor((2, 2, 2, 2), 3, nrhs=2))
