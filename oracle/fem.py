"""Finite elements of the elastic scatterer and the BEM-FEM coupled operator.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.3 discretises the weak form of the elastic body (Eq. fem_2: the
pressure load on the boundary, the stiffness and the inertia terms) with
linear tetrahedra and couples it to the collocation BEM (Eq. renritupu);
eliminating the displacement gives the Schur form (Eqs. kousokuu, GMRES).
Plain dense float64 / complex128 throughout.

Readings (the paper fixes the element types, not the signs or the normal):
* n is the unit normal of the boundary triangles pointing into the fluid
  (out of the body), as for the BEM; the traction of the fluid on the body
  is -p n, so the load vector is -N p with N[3a+i, j] = int_{Gamma_j} phi_a n_i
  = A_j n_{j,i} / 3 (p constant on triangle j, phi_a linear);
* the normal derivative of the pressure on the fluid side follows from the
  momentum balance (time factor exp(-i omega t)): dp/dn = rho_f omega^2 u.n;
  per triangle it is taken at the collocation point, where the linear u
  equals its mean over the triangle: q_j = rho_f omega^2 n_j . (u_a+u_b+u_c)/3;
* hence q = C p with C = -rho_f omega^2 Tc (K - omega^2 M)^(-1) N,
  Tc[j, 3a+i] = n_{j,i} / 3, and the coupled operator is Mp + Mq C with the
  BEM blocks of the product (I/2 - K - alpha H, S + alpha K' + alpha/2 I);
  alpha = 0 is the paper's Eq. GMRES.
"""
import numpy as np


def tet_geometry(X):
    """Signed volume and gradients of the four barycentric (linear shape)
    functions of the tetrahedron with vertices X (4 x 3)."""
    J = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)   # columns
    vol = np.linalg.det(J) / 6.0
    Ji = np.linalg.inv(J)                 # rows: gradients of phi_1, phi_2, phi_3
    g = np.vstack([-Ji.sum(axis=0), Ji])
    return vol, g


def elasticity_matrices(nodes, tets, lam, mu, rho):
    """Dense stiffness K and consistent mass M (3n x 3n, dof 3a + i) of an
    isotropic body: K_e[(a,i),(b,j)] = V (lam d_i phi_a d_j phi_b
    + mu (delta_ij grad phi_a . grad phi_b + d_j phi_a d_i phi_b)),
    M_e[(a,i),(b,j)] = delta_ij rho V (1 + delta_ab) / 20."""
    n = len(nodes)
    K = np.zeros((3 * n, 3 * n))
    M = np.zeros((3 * n, 3 * n))
    for t in tets:
        vol, g = tet_geometry(nodes[t])
        V = abs(vol)
        dof = (3 * np.asarray(t)[:, None] + np.arange(3)[None, :]).ravel()
        Ke = np.zeros((12, 12))
        Me = np.zeros((12, 12))
        for a in range(4):
            for b in range(4):
                blk = lam * np.outer(g[a], g[b]) + mu * (np.dot(g[a], g[b]) * np.eye(3)
                                                         + np.outer(g[b], g[a]))
                Ke[3 * a:3 * a + 3, 3 * b:3 * b + 3] = V * blk
                Me[3 * a:3 * a + 3, 3 * b:3 * b + 3] = rho * V * (2.0 if a == b else 1.0) / 20 * np.eye(3)
        K[np.ix_(dof, dof)] += Ke
        M[np.ix_(dof, dof)] += Me
    return K, M


def surface_coupling(nodes, T):
    """Tc (n_tri x 3n) and N (3n x n_tri): Tc[j, 3a+i] = n_{j,i}/3 for the
    vertices a of triangle j, N = Tc^T diag(area); also area and normal."""
    n = len(nodes)
    X = nodes[T]
    c = np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0])
    area = 0.5 * np.linalg.norm(c, axis=1)
    nrm = c / (2 * area)[:, None]
    Tc = np.zeros((len(T), 3 * n))
    for j, tri in enumerate(T):
        for a in tri:
            Tc[j, 3 * a:3 * a + 3] += nrm[j] / 3.0
    return Tc, Tc.T * area[None, :], area, nrm


def coupling_matrix(nodes, tets, T, lam, mu, rho_s, rho_f, omega):
    """C = -rho_f omega^2 Tc (K - omega^2 M)^(-1) N (n_tri x n_tri, real):
    q = C p is the normal derivative of the pressure that the body's
    response to the boundary pressure p produces (Eq. kousokuu)."""
    K, M = elasticity_matrices(nodes, tets, lam, mu, rho_s)
    Tc, N, _, _ = surface_coupling(nodes, T)
    X = np.linalg.solve(K - omega ** 2 * M, N)
    return -rho_f * omega ** 2 * (Tc @ X)


def coupled_operator(Mp, Mq, C):
    """The Schur form of the coupled system: Mp + Mq C (Eq. GMRES)."""
    return Mp + Mq @ C
