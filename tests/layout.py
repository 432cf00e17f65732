"""Test helpers: move vectors between the oracle numbering and the library's
padded SoA layout, and seeded inputs.  Holds none of the method's arithmetic.

Padded layout: block of P = (Nx+2)(Ny+2)(Nz+2) per component, element
(i,j,k) at (i+1) + (Nx+2)((j+1) + (Ny+2)(k+1)) -- i.e. a C-ordered array of
shape (Nz+2, Ny+2, Nx+2) indexed [k+1, j+1, i+1].  The oracle stores each
face family as a C-ordered array [k, j, i] of its own shape.
"""
import numpy as np

FACE_SHAPES = (lambda n: (n[2], n[1], n[0] + 1),
               lambda n: (n[2], n[1] + 1, n[0]),
               lambda n: (n[2] + 1, n[1], n[0]))
EDGE_SHAPES = (lambda n: (n[2] + 1, n[1] + 1, n[0]),
               lambda n: (n[2] + 1, n[1], n[0] + 1),
               lambda n: (n[2], n[1] + 1, n[0] + 1))


def pshape(n):
    return (n[2] + 2, n[1] + 2, n[0] + 2)


def padded_size(n):
    return int(np.prod(pshape(n)))


def to_padded(arr, n):
    """One oracle family array [k, j, i] -> flat padded block."""
    out = np.zeros(pshape(n))
    s = arr.shape
    out[1:1 + s[0], 1:1 + s[1], 1:1 + s[2]] = arr
    return out.ravel()


def from_padded(block, n, shape):
    a = np.asarray(block).reshape(pshape(n))
    return a[1:1 + shape[0], 1:1 + shape[1], 1:1 + shape[2]].copy()


def faces_to_padded(full_vec, n):
    """Oracle full face vector (x-, y-, z-families) -> padded 3P vector."""
    out = []
    off = 0
    for a in range(3):
        shp = FACE_SHAPES[a](n)
        m = int(np.prod(shp))
        out.append(to_padded(full_vec[off:off + m].reshape(shp), n))
        off += m
    return np.concatenate(out)


def faces_from_padded(vec, n):
    P = padded_size(n)
    parts = [from_padded(vec[a * P:(a + 1) * P], n, FACE_SHAPES[a](n)).ravel() for a in range(3)]
    return np.concatenate(parts)


def cells_to_padded(vec, n):
    return to_padded(np.asarray(vec).reshape(n[2], n[1], n[0]), n)


def cells_from_padded(vec, n):
    return from_padded(vec, n, (n[2], n[1], n[0])).ravel()


def fractions_to_padded(fr, n):
    """Oracle fraction dict -> (7, P) array ax ay az lx ly lz v."""
    rows = [to_padded(fr[s], n) for s in ("ax", "ay", "az", "lx", "ly", "lz", "v")]
    return np.stack(rows)


def fractions_from_padded(fr7, n):
    names = ("ax", "ay", "az", "lx", "ly", "lz", "v")
    shapes = [FACE_SHAPES[0](n), FACE_SHAPES[1](n), FACE_SHAPES[2](n),
              EDGE_SHAPES[0](n), EDGE_SHAPES[1](n), EDGE_SHAPES[2](n), (n[2], n[1], n[0])]
    return {s: from_padded(fr7[q], n, shp) for q, (s, shp) in enumerate(zip(names, shapes))}


def random_active(op_oracle, seed):
    """Seeded N(0,1) vector on the oracle's active faces."""
    return np.random.default_rng(seed).standard_normal(op_oracle.act.size)
