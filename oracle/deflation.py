"""Crack-aware deflation of the elastic solve (the possible improvement
named at the end of Sec. 3.1, the linear elastic subproblem).

Test infrastructure (see the package docstring).

Sec. 3.1 observes that once damage splits the body into undamaged pieces, the
elastic operator acquires extra near-null vectors: the rigid motions of each
piece, whose energy is carried only by the residual stiffness k_ell of the
damaged band (or by whatever Dirichlet condition the piece touches).  The
paper supplies only the rigid modes of the whole body to its multigrid and
names approximating the per-piece modes as a possible improvement.  The
reading implemented here:

* Fragments: connected components of the undamaged nodes {alpha < theta}
  in the graph of the mesh's element edges.  A component is named by its
  smallest node index.  Components of fewer than ``min_nodes`` nodes are
  dropped; of the rest, at most ``max_fragments`` are kept, the largest
  first, ties by the smaller name.
* Coarse space W: for each kept fragment, its three 2D rigid modes -- the
  x and y translations and the rotation (-(y - yc), x - xc) * s about the
  domain centre (xc, yc) = (lx/2, ly/2), s = 2 / max(lx, ly) -- restricted
  to the fragment's nodes and set to zero on Dirichlet DOFs, so that every
  column lies in the space the elastic solve searches.
* E = W^T K W, and deflated CG in the form of Saad, Yeung, Erhel and
  Guyomarc'h (2000): start x0 = x + W E^{-1} W^T (b - K x); directions
  p = z + beta p - W E^{-1} W^T K z, so that W^T r = 0 at every iterate.

``fragments`` walks the element edges by breadth-first search in plain
Python (small meshes only).
"""

from collections import deque

import numpy as np


def _adjacency(T, N):
    adj = [set() for _ in range(N)]
    for tri in T:
        for a in range(len(tri)):
            for b in range(a + 1, len(tri)):
                u, v = int(tri[a]), int(tri[b])
                adj[u].add(v)
                adj[v].add(u)
    return adj


def components(T, N, solid):
    """Name (smallest node index) of each solid node's component, -1 for the
    others; components of the graph of element edges between solid nodes."""
    adj = _adjacency(T, N)
    name = np.full(N, -1, dtype=np.int64)
    for s in range(N):
        if not solid[s] or name[s] >= 0:
            continue
        # s is the smallest unvisited solid node, hence its component's minimum
        name[s] = s
        todo = deque([s])
        while todo:
            u = todo.popleft()
            for v in adj[u]:
                if solid[v] and name[v] < 0:
                    name[v] = s
                    todo.append(v)
    return name


def fragments(T, N, alpha, theta=0.5, min_nodes=64, max_fragments=8):
    """(fid, roots): fragment index of every node (-1: damaged or in a
    dropped component) and the kept components' names in fragment order."""
    name = components(T, N, np.asarray(alpha) < theta)
    roots, sizes = np.unique(name[name >= 0], return_counts=True)
    keep = [(-int(c), int(r)) for r, c in zip(roots, sizes) if c >= min_nodes]
    keep.sort()
    kept = [r for _, r in keep[:max_fragments]]
    fid = np.full(N, -1, dtype=np.int64)
    for k, r in enumerate(kept):
        fid[name == r] = k
    return fid, kept


def rigid_modes(X, fixed, fid, nfrag, lx, ly):
    """W [2N, 3 nfrag]: per fragment the x and y translations and the scaled
    rotation about the domain centre, zero off the fragment and on fixed
    DOFs (component-major DOFs [u_x | u_y])."""
    N = X.shape[0]
    xc, yc, s = 0.5 * lx, 0.5 * ly, 2.0 / max(lx, ly)
    W = np.zeros((2 * N, 3 * nfrag))
    for f in range(nfrag):
        on = fid == f
        W[:N, 3 * f][on] = 1.0
        W[N:, 3 * f + 1][on] = 1.0
        W[:N, 3 * f + 2][on] = -(X[on, 1] - yc) * s
        W[N:, 3 * f + 2][on] = (X[on, 0] - xc) * s
    W[fixed, :] = 0.0
    return W


def coarse_matrix(K, W):
    """E = W^T K W."""
    return W.T @ (K @ W)


def deflated_cg(K, b, x, W, tol, maxit=10000, Minv=None):
    """Deflated (preconditioned) CG on K x = b from x.  Returns
    (x, iterations, max_k |W^T r_k| / |b|).  Minv: the preconditioner as a
    function (identity when None)."""
    Einv = np.linalg.inv(coarse_matrix(K, W)) if W.shape[1] else np.zeros((0, 0))
    M = Minv if Minv is not None else (lambda v: v)

    def project(v):                     # W E^{-1} W^T v
        return W @ (Einv @ (W.T @ v))

    r = b - K @ x
    x = x + project(r)
    r = b - K @ x
    bn = max(np.linalg.norm(b), 1e-300)
    worst = np.max(np.abs(W.T @ r)) / bn if W.shape[1] else 0.0
    if np.linalg.norm(r) <= tol:
        return x, 0, worst
    z = M(r)
    p = z - project(K @ z)
    rz = r @ z
    for it in range(1, maxit + 1):
        q = K @ p
        a = rz / (p @ q)
        x = x + a * p
        r = r - a * q
        if W.shape[1]:
            worst = max(worst, np.max(np.abs(W.T @ r)) / bn)
        if np.linalg.norm(r) <= tol:
            return x, it, worst
        z = M(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p - project(K @ z)
        rz = rz_new
    return x, maxit, worst
