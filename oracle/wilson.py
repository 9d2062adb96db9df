"""The 2D Wilson-Dirac matrix, written out entry by entry (paper, Introduction).

The paper defines, for d dimensions,

    D_{x,y} = -1/2 sum_mu [ (1 - gamma_mu) U_x^mu delta_{x+mu,y}
                           + (1 + gamma_mu) U_{x-mu}^{mu*} delta_{x-mu,y} ] + (2d + m) delta_{x,y}

Readings taken here (each is listed with its reason in the design notes):

* d = 2 with the Pauli matrices gamma_x = sigma1, gamma_t = sigma2 (two spin
  components per site; gamma5 = sigma3).
* Diagonal term (d + m) = (2 + m): the standard Wilson normalisation in which the
  free operator at zero momentum equals m.  The literal (2d + m) is the same
  operator at the shifted mass m + 2.
* Fermion boundary condition periodic in x and antiperiodic in t, realised by
  flipping the sign of the t-links on the last time slice inside the operator
  only (plaquettes and the topological charge are unchanged).

Indexing: site s = t*lx + x; vector index i = 2*s + spin; gauge links U[mu, t, x].
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

SIGMA1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SIGMA2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SIGMA3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
GAMMA = (SIGMA1, SIGMA2)
ID2 = np.eye(2, dtype=np.complex128)


def fermion_links(U: np.ndarray, antiperiodic_t: bool = True) -> np.ndarray:
    """Links seen by the fermion: U with the t-links of the last slice negated."""
    Ut = np.array(U, dtype=np.complex128, copy=True)
    if antiperiodic_t:
        Ut[1, -1, :] *= -1.0
    return Ut


def _block_triplets(rows_site, cols_site, coef, M):
    """COO triplets for the 2x2 blocks coef[s] * M placed at (rows_site[s], cols_site[s])."""
    r, c, v = [], [], []
    for a in range(2):
        for b in range(2):
            if M[a, b] == 0:
                continue
            r.append(2 * rows_site + a)
            c.append(2 * cols_site + b)
            v.append(coef * M[a, b])
    return r, c, v


def dirac_matrix(U: np.ndarray, mass: float, antiperiodic_t: bool = True) -> sp.csr_matrix:
    """Sparse D (complex128, shape [2V, 2V]) for gauge links U[2, lt, lx]."""
    _, lt, lx = U.shape
    V = lx * lt
    Ut = fermion_links(U, antiperiodic_t)
    t, x = np.meshgrid(np.arange(lt), np.arange(lx), indexing="ij")
    s = (t * lx + x).ravel()
    rows, cols, vals = [], [], []
    # Diagonal (2 + m).
    r, c, v = _block_triplets(s, s, np.full(V, 2.0 + mass, dtype=np.complex128), ID2)
    rows += r; cols += c; vals += v
    for mu in range(2):
        if mu == 0:
            fwd = (t * lx + (x + 1) % lx).ravel()
            bwd = (t * lx + (x - 1) % lx).ravel()
            link_bwd = Ut[0][t, (x - 1) % lx].ravel()
        else:
            fwd = (((t + 1) % lt) * lx + x).ravel()
            bwd = (((t - 1) % lt) * lx + x).ravel()
            link_bwd = Ut[1][(t - 1) % lt, x].ravel()
        link_fwd = Ut[mu].ravel()
        g = GAMMA[mu]
        r, c, v = _block_triplets(s, fwd, -0.5 * link_fwd, ID2 - g)
        rows += r; cols += c; vals += v
        r, c, v = _block_triplets(s, bwd, -0.5 * np.conj(link_bwd), ID2 + g)
        rows += r; cols += c; vals += v
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.coo_matrix((vals, (rows, cols)), shape=(2 * V, 2 * V)).tocsr()


def dirac_dagger(U: np.ndarray, mass: float, antiperiodic_t: bool = True) -> sp.csr_matrix:
    """D^H, the literal conjugate transpose of D."""
    return dirac_matrix(U, mass, antiperiodic_t).conj().T.tocsr()


def normal_matrix(U: np.ndarray, mass: float, antiperiodic_t: bool = True) -> sp.csr_matrix:
    """A = D^H D, the Hermitian positive definite operator the multigrid acts on."""
    D = dirac_matrix(U, mass, antiperiodic_t)
    return (D.conj().T @ D).tocsr()


def gamma5_matrix(V: int) -> sp.csr_matrix:
    """sigma3 acting on every site (gamma5 in two dimensions)."""
    return sp.kron(sp.identity(V, format="csr"), sp.csr_matrix(SIGMA3)).tocsr()
