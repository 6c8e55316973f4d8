"""Independent dense brute-force route for tiny meshes (test infrastructure only).

It rebuilds the screened Poisson matrix A = Z^T (D^T G D + lambda C) Z of
arXiv:2202.12477 (NekBone section, eq. poisson and eq. stiffness) by a route
that shares nothing with ``oracle.c`` beyond the vertex coordinates it is given:

- GLL nodes: roots of P_N' from numpy's Legendre module (eigenvalues of a
  companion matrix), weights 2/(N(N+1)P_N^2);
- D: l_j'(xi_i) from a Legendre Vandermonde matrix, D = V_r V^{-1};
- the Jacobian: D applied to the nodal coordinates of the trilinear map (the
  map is in Q1, a subspace of Q_N, so this is exact);
- the gradient and divergence: explicit Kronecker products (numpy.kron);
- Z: a dense 0/1 matrix from the global numbering.

Also the closed form of an affine (undistorted) box: A = K(x)M(x)M + M(x)K(x)M +
M(x)M(x)K + lambda M(x)M(x)M with assembled 1D stiffness K and diagonal mass M,
applied by three 1D contractions.  Cost O(N_G (nN+1)), usable at any size.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as L


def gll(N: int):
    cN = np.zeros(N + 1)
    cN[N] = 1.0
    interior = np.sort(np.real(L.legroots(L.legder(cN)))) if N >= 2 else np.array([])
    xi = np.concatenate([[-1.0], interior, [1.0]])
    w = 2.0 / (N * (N + 1) * L.legval(xi, cN) ** 2)
    return xi, w


def deriv(N: int, xi: np.ndarray) -> np.ndarray:
    V = np.stack([L.legval(xi, np.eye(N + 1)[k]) for k in range(N + 1)], axis=1)
    Vr = np.stack([L.legval(xi, L.legder(np.eye(N + 1)[k])) for k in range(N + 1)], axis=1)
    return Vr @ np.linalg.inv(V)


def global_ids(nx, ny, nz, N):
    """Z as an index array [E, Np]: local (a,b,c) of element (ex,ey,ez)."""
    n1 = N + 1
    gx, gy = nx * N + 1, ny * N + 1
    ids = np.empty((nx * ny * nz, n1 ** 3), dtype=np.int64)
    a = np.arange(n1)
    A, B, C = np.meshgrid(a, a, a, indexing="ij")  # A[a,b,c]
    loc = (A + n1 * (B + n1 * C)).ravel()
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                e = ex + nx * (ey + ny * ez)
                g = (ex * N + A) + gx * ((ey * N + B) + gy * (ez * N + C))
                ids[e, loc] = g.ravel()
    return ids


def dense_matrix(nx, ny, nz, N, V: np.ndarray, lam: float, mass: int = 0) -> np.ndarray:
    """Dense assembled A for a box of nx*ny*nz elements with vertices V[(nx+1)(ny+1)(nz+1), 3]."""
    n1 = N + 1
    Np = n1 ** 3
    xi, w = gll(N)
    D = deriv(N, xi)
    I = np.eye(n1)
    # local index a + n1*(b + n1*c): a is the fastest, so it is the last Kronecker factor
    Dr = np.kron(I, np.kron(I, D))
    Ds = np.kron(I, np.kron(D, I))
    Dt = np.kron(D, np.kron(I, I))
    W3 = np.kron(w, np.kron(w, w))  # w_c w_b w_a in local order
    ids = global_ids(nx, ny, nz, N)
    NG = (nx * N + 1) * (ny * N + 1) * (nz * N + 1)
    mult = np.bincount(ids.ravel(), minlength=NG)
    A = np.zeros((NG, NG))
    # trilinear basis values at the GLL nodes: phi_corner(xi) per axis
    phi = np.stack([(1 - xi) / 2, (1 + xi) / 2])  # [corner bit, node]
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                e = ex + nx * (ey + ny * ez)
                X = np.zeros((Np, 3))
                for dz in range(2):
                    for dy in range(2):
                        for dx in range(2):
                            v = (ex + dx) + (nx + 1) * ((ey + dy) + (ny + 1) * (ez + dz))
                            weight = np.kron(phi[dz], np.kron(phi[dy], phi[dx]))
                            X += np.outer(weight, V[v])
                # Jm[n, i, d] = d x_i / d xi_d, by the derivative matrix on nodal coordinates
                Jm = np.stack([Dr @ X, Ds @ X, Dt @ X], axis=2)
                J = np.linalg.det(Jm)
                R = np.linalg.inv(Jm)  # R[n, d, i] = d xi_d / d x_i
                Gm = np.einsum("ndi,nei->nde", R, R) * (W3 * J)[:, None, None]
                grad = np.stack([Dr, Ds, Dt])  # [d, node, node]
                Se = np.einsum("dnm,nde,enk->mk", grad, Gm, grad)
                c = W3 * J if mass == 0 else 1.0 / mult[ids[e]]
                Ae = Se + lam * np.diag(c)
                Z = np.zeros((Np, NG))
                Z[np.arange(Np), ids[e]] = 1.0
                A += Z.T @ Ae @ Z
    return A


def assembled_1d(n: int, N: int):
    """Assembled 1D stiffness K and diagonal mass M on [0,1] with n equal elements."""
    xi, w = gll(N)
    D = deriv(N, xi)
    h = 1.0 / n
    Khat = D.T @ np.diag(w) @ D
    m = n * N + 1
    K = np.zeros((m, m))
    M = np.zeros(m)
    for e in range(n):
        s = slice(e * N, e * N + N + 1)
        K[s, s] += (2.0 / h) * Khat
        M[s] += (h / 2.0) * w
    return K, M


def affine_box_ax(nx, ny, nz, N, lam: float, x: np.ndarray) -> np.ndarray:
    """A x on an affine unit box via its Kronecker closed form (mass = GLL weight x J)."""
    Kx, Mx = assembled_1d(nx, N)
    Ky, My = assembled_1d(ny, N)
    Kz, Mz = assembled_1d(nz, N)
    X = x.reshape(nz * N + 1, ny * N + 1, nx * N + 1)  # [K, J, I]
    Mzb, Myb, Mxb = Mz[:, None, None], My[None, :, None], Mx[None, None, :]
    Y = (Mzb * Myb) * (X @ Kx)                       # K along x
    Y += Mzb * Mxb * np.einsum("jl,kli->kji", Ky, X)  # K along y
    Y += Myb * Mxb * np.einsum("kl,lji->kji", Kz, X)  # K along z
    Y += lam * (Mzb * Myb * Mxb) * X
    return Y.ravel()
