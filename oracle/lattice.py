"""Lattice index space, shifts and the x0 block decomposition (oracle).

Sec. 1: sites x = (x0, x1, x2, x3), 0 <= x_i < L_i, directions mu in {0,1,2,3}.
Fields carry the four lattice axes followed by exactly two inner axes (spin x colour for a
spinor, row x colour for one link direction), optionally preceded by batch axes, so the
lattice axis of direction mu is ``ndim - 6 + mu``.

Boundary conditions (the paper states none): gauge links periodic in all directions;
fermion hops periodic in space and antiperiodic in x0, i.e. a hop that wraps around the
x0 boundary carries a factor -1.

Blocks (Sec. 1, one-dimensional decomposition): l_mu = L_mu for mu = 1,2,3, so block b
holds the slices b*l0 <= x0 < (b+1)*l0. Red/black colouring: black = odd block index
(the paper leaves the choice open; det R does not depend on it).
"""
import numpy as np


def lattice_axis(f: np.ndarray, mu: int) -> int:
    return f.ndim - 6 + mu


def shift_fwd(f: np.ndarray, mu: int, fermion: bool) -> np.ndarray:
    """g(x) = f(x + mu^); with ``fermion`` the x0 wrap picks up a factor -1."""
    ax = lattice_axis(f, mu)
    g = np.roll(f, -1, axis=ax)
    if fermion and mu == 0:
        idx = [slice(None)] * f.ndim
        idx[ax] = -1                     # sites x0 = L0-1 read f at x0 = 0 through the wrap
        g[tuple(idx)] *= -1.0
    return g


def shift_bwd(f: np.ndarray, mu: int, fermion: bool) -> np.ndarray:
    """g(x) = f(x - mu^); with ``fermion`` the x0 wrap picks up a factor -1."""
    ax = lattice_axis(f, mu)
    g = np.roll(f, 1, axis=ax)
    if fermion and mu == 0:
        idx = [slice(None)] * f.ndim
        idx[ax] = 0                      # sites x0 = 0 read f at x0 = L0-1 through the wrap
        g[tuple(idx)] *= -1.0
    return g


def coords(L):
    """Integer coordinate arrays x0, x1, x2, x3 of shape L."""
    return np.meshgrid(*[np.arange(n) for n in L], indexing="ij")


def parity(L) -> np.ndarray:
    """(x0 + x1 + x2 + x3) mod 2: 0 = even, 1 = odd."""
    x = coords(L)
    return (x[0] + x[1] + x[2] + x[3]) % 2


def block_of_x0(x0, l0: int):
    return np.asarray(x0) // l0


def site_mask(L, where) -> np.ndarray:
    """Boolean mask of shape L broadcastable onto a spinor field (adds two inner axes)."""
    return np.asarray(where, dtype=bool)[..., None, None]


def colour_x0_mask(L, l0: int, colour: str) -> np.ndarray:
    """Sites whose x0 block has the given colour: 'all', 'black' (odd b) or 'white'."""
    x0 = coords(L)[0]
    b = block_of_x0(x0, l0)
    if colour == "all":
        m = np.ones(L, dtype=bool)
    elif colour == "black":
        m = (b % 2) == 1
    elif colour == "white":
        m = (b % 2) == 0
    else:
        raise ValueError(colour)
    return m


def single_block_mask(L, l0: int, block: int) -> np.ndarray:
    x0 = coords(L)[0]
    return block_of_x0(x0, l0) == block
