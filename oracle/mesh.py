"""Structured simplicial meshes for the P1 discretisation (Sec. 1.2).

The paper discretises with P1 Lagrange elements on simplicial meshes.  The
workloads used here are structured:

* 2D: an nx-by-ny grid of rectangular cells, each split along its diagonal
  from the lower-left to the upper-right corner ("right-diagonal").
* 3D: an nx-by-ny-by-nz grid of hexahedra, each split into the six Kuhn
  tetrahedra that share the hexahedron's main diagonal.

Node numbering (shared by every consumer of these meshes, so vectors can be
compared entry by entry): node (i, j[, k]) has id i + (nx+1)*(j + (ny+1)*k).
A displacement vector stores component c of node n at c*N + n ("blocked").
"""

import itertools

import numpy as np


def node_id_2d(i, j, nx):
    return i + (nx + 1) * j


def node_id_3d(i, j, k, nx, ny):
    return i + (nx + 1) * (j + (ny + 1) * k)


def structured_mesh_2d(nx, ny, lx=1.0, ly=1.0):
    """Nodes X[N,2] and triangles T[2*nx*ny,3].

    Cell (i, j) yields, in this order, the triangles
    [(i,j), (i+1,j), (i+1,j+1)] and [(i,j), (i+1,j+1), (i,j+1)];
    element index 2*(i + nx*j) + t.
    """
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="xy")
    X = np.stack([ii.ravel() * (lx / nx), jj.ravel() * (ly / ny)], axis=1).astype(np.float64)
    ci, cj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    ci = ci.ravel()
    cj = cj.ravel()
    n00 = node_id_2d(ci, cj, nx)
    n10 = node_id_2d(ci + 1, cj, nx)
    n11 = node_id_2d(ci + 1, cj + 1, nx)
    n01 = node_id_2d(ci, cj + 1, nx)
    T = np.empty((2 * nx * ny, 3), dtype=np.int64)
    T[0::2] = np.stack([n00, n10, n11], axis=1)
    T[1::2] = np.stack([n00, n11, n01], axis=1)
    return X, T


def kuhn_permutations():
    """The 6 axis orderings; tetrahedron p has vertices v0, v0+e_p0,
    v0+e_p0+e_p1, v0+(1,1,1)."""
    return list(itertools.permutations(range(3)))


def structured_mesh_3d(nx, ny, nz, lx=1.0, ly=1.0, lz=1.0):
    """Nodes X[N,3] and Kuhn tetrahedra T[6*nx*ny*nz,4].

    Hexahedron (i, j, k) yields 6 tetrahedra, one per permutation p of the
    axes (in ``itertools.permutations`` order); element index
    6*(i + nx*(j + ny*k)) + p.
    """
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    # order nodes with i fastest, then j, then k
    ii = ii.transpose(2, 1, 0).ravel()
    jj = jj.transpose(2, 1, 0).ravel()
    kk = kk.transpose(2, 1, 0).ravel()
    X = np.stack([ii * (lx / nx), jj * (ly / ny), kk * (lz / nz)], axis=1).astype(np.float64)
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()
    perms = kuhn_permutations()
    T = np.empty((len(ci) * 6, 4), dtype=np.int64)
    for p, perm in enumerate(perms):
        off = np.zeros((4, 3), dtype=np.int64)
        off[1, perm[0]] = 1
        off[2] = off[1]
        off[2, perm[1]] = 1
        off[3] = 1
        for v in range(4):
            T[p::6, v] = node_id_3d(ci + off[v, 0], cj + off[v, 1], ck + off[v, 2], nx, ny)
    return X, T
