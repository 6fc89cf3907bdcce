"""Oracle: explicit collocation matrix A(E) = H - E S and the separable block.

Test infrastructure only (see oracle/__init__.py).

H is the collocation discretisation of eq. (FM-pre) with the right-hand side
moved to the left and E = 0 (Sec. 3.1: H c = E S c, collocation matrix H of
the operator, S the basis-at-points matrix; Sec. 3.3: H = L~ + R~).  Every row
belongs to one collocation point (alpha, M', zeta, xi, eta) and every column to
one basis product S^k(z) S^i(x) S^j(y) of component (beta, M''); an entry is
the operator applied to that product and evaluated at that point:

  diagonal in (alpha, M'), from the hatted kinetic operator and potentials:
      - S_j''(y) - S_i''(x) - (1/x^2 + 1/y^2)[(1-z^2) S_k'' - 2(M'+1) z S_k' - M'(M'+1) S_k]
      + [(J(J+1) - 2M'^2)/y^2 + V_a(x) + sum_{b != a} V_b^(l)(x_b, y_b) - E] S_k S_i S_j
  (alpha, M') <- (alpha, M'+1): lambda-hat^{J,M'} y^-2 [-(1-z^2) S_k' + 2(M'+1) z S_k] S_i S_j
  (alpha, M') <- (alpha, M'-1): lambda-hat^{J,-M'} y^-2 S_k' S_i S_j
  (alpha, M') <- (beta, M''), beta != alpha, the rearrangement (coupling) term:
      + V_a^(s)(x, y) (x y / (x_b y_b)) (1-z_b^2)^{M''/2} / (1-z^2)^{M'/2}
        (-1)^{M''-M'} 2/sqrt(2+2 delta_{M''0}) F^{J tau}_{M''M'}(0, w_ba, 0)
        S^k_b(z_b) S^i_b(x_b) S^j_b(y_b),
      with the beta expansion taken as zero outside beta's box (bound-state
      Dirichlet condition).

The coupling enters with a plus sign: eq. (FM-pre) has it on the right with a
minus sign, and H is the left side minus the right side.

Unknowns and rows are ordered [alpha][M'][z][x][y] (y fastest, Sec. 3.2).
"""
import math

import numpy as np
import scipy.sparse as sp

from . import physics as ph
from .basis import basis_for
from .wigner import F_rot, lam_hat_minus, lam_hat_plus, w_angle


class Problem:
    def __init__(self, desc):
        self.desc = desc
        self.J, self.tau = desc["J"], desc["tau"]
        if self.tau not in (1, -1) or self.J < 0:
            raise ValueError("bad J / tau")
        self.M0 = (1 - self.tau) // 2
        self.Mps = list(range(self.M0, self.J + 1))
        self.nM = len(self.Mps)
        if self.nM < 1:
            raise ValueError("no M' blocks")
        self.bx = [basis_for(desc["x"][a], "xy") for a in range(3)]
        self.by = [basis_for(desc["y"][a], "xy") for a in range(3)]
        self.bz = [basis_for(desc["z"][a], "z") for a in range(3)]
        self.block = [self.bz[a].n * self.bx[a].n * self.by[a].n for a in range(3)]
        self.offsets = []
        off = 0
        for a in range(3):
            row = []
            for _ in range(self.nM):
                row.append(off)
                off += self.block[a]
            self.offsets.append(row)
        self.N = off

    # -- index helpers ------------------------------------------------------
    def split_index(self, g):
        """Global index -> (alpha, iM, zeta, xi, eta)."""
        for a in range(3):
            for iM in range(self.nM):
                o = self.offsets[a][iM]
                if o <= g < o + self.block[a]:
                    l = g - o
                    nx, ny = self.bx[a].n, self.by[a].n
                    return a, iM, l // (nx * ny), (l // ny) % nx, l % ny
        raise IndexError(g)

    def points(self, a):
        bz, bx, by = self.bz[a], self.bx[a], self.by[a]
        Z, X, Y = np.meshgrid(bz.points, bx.points, by.points, indexing="ij")
        return Z.ravel(), X.ravel(), Y.ravel()

    # -- rows -----------------------------------------------------------------
    def _rows(self, a, iM, sel, E):
        """Triplets (local_row, col, val) of the rows of block (a, M') at the
        local point indices sel (zeta*nx*ny + xi*ny + eta)."""
        d = self.desc
        J, Mp = self.J, self.Mps[iM]
        bz, bx, by = self.bz[a], self.bx[a], self.by[a]
        nx, ny = bx.n, by.n
        zeta, xi, eta = sel // (nx * ny), (sel // ny) % nx, sel % ny
        z, x, y = bz.points[zeta], bx.points[xi], by.points[eta]
        P = ph.potential_field(d, a, x, y, z)

        iz, Sz = bz.local(z, 0)
        _, D1z = bz.local(z, 1)
        _, D2z = bz.local(z, 2)
        ix, Sx = bx.local(x, 0)
        _, D2x = bx.local(x, 2)
        iy, Sy = by.local(y, 0)
        _, D2y = by.local(y, 2)

        inv2 = (1.0 / x ** 2 + 1.0 / y ** 2)[:, None]
        dz = ((1 - z * z)[:, None] * D2z - 2 * (Mp + 1) * z[:, None] * D1z - Mp * (Mp + 1) * Sz)
        diagc = ((J * (J + 1) - 2 * Mp * Mp) / y ** 2 + P - E)

        out_r, out_c, out_v = [], [], []

        def emit(b, jM, izz, ixx, iyy, V):
            """Add the entries V[p, kz, kx, ky] of column block (b, M'') for the
            local basis indices izz[p, kz], ixx[p, kx], iyy[p, ky] (-1: dropped)."""
            nxb, nyb = self.bx[b].n, self.by[b].n
            valid = (izz[:, :, None, None] >= 0) & (ixx[:, None, :, None] >= 0) & (iyy[:, None, None, :] >= 0)
            cols = (self.offsets[b][jM] + (izz[:, :, None, None] * nxb + ixx[:, None, :, None]) * nyb
                    + iyy[:, None, None, :])
            rows = np.broadcast_to(np.arange(sel.size)[:, None, None, None], V.shape)
            m = valid & (V != 0.0)
            out_r.append(rows[m])
            out_c.append(cols[m])
            out_v.append(V[m])

        # diagonal block (alpha, M')
        V = (-Sz[:, :, None, None] * Sx[:, None, :, None] * D2y[:, None, None, :]
             - Sz[:, :, None, None] * D2x[:, None, :, None] * Sy[:, None, None, :]
             - inv2[:, :, None, None] * dz[:, :, None, None] * Sx[:, None, :, None] * Sy[:, None, None, :]
             + diagc[:, None, None, None] * Sz[:, :, None, None] * Sx[:, None, :, None] * Sy[:, None, None, :])
        emit(a, iM, iz, ix, iy, V)

        # M' +- 1 kinetic couplings
        if iM + 1 < self.nM:
            f = lam_hat_plus(J, Mp) / y ** 2
            zp = -(1 - z * z)[:, None] * D1z + 2 * (Mp + 1) * z[:, None] * Sz
            V = f[:, None, None, None] * zp[:, :, None, None] * Sx[:, None, :, None] * Sy[:, None, None, :]
            emit(a, iM + 1, iz, ix, iy, V)
        if iM - 1 >= 0:
            f = lam_hat_minus(J, Mp) / y ** 2
            V = f[:, None, None, None] * D1z[:, :, None, None] * Sx[:, None, :, None] * Sy[:, None, None, :]
            emit(a, iM - 1, iz, ix, iy, V)

        # coupling to the other components
        vs = ph.v_short(d, a, x, y)
        for b in ph.others(a):
            c, s = ph.rotation_cs(d["masses"], b, a)
            xb, yb, zb = ph.rotated_coords(x, y, z, c, s)
            inside = (xb <= self.bx[b].R) & (yb <= self.by[b].R)
            if not np.any(inside):
                continue
            jz, Tz = self.bz[b].local(zb, 0)
            jx, Tx = self.bx[b].local(np.minimum(xb, self.bx[b].R), 0)
            jy, Ty = self.by[b].local(np.minimum(yb, self.by[b].R), 0)
            base = np.where(inside, vs * x * y / (xb * yb), 0.0)
            prod = Tz[:, :, None, None] * Tx[:, None, :, None] * Ty[:, None, None, :]
            w = w_angle(d["masses"], b, a, x, y, z, yb) if self.J > 0 else None
            for jM, Mpp in enumerate(self.Mps):
                if self.J == 0:
                    f = base
                else:
                    f = (base * (1 - zb * zb) ** (Mpp / 2.0) / (1 - z * z) ** (Mp / 2.0)
                         * (-1.0) ** (Mpp - Mp) * 2.0 / math.sqrt(2.0 + 2.0 * (Mpp == 0))
                         * F_rot(J, self.tau, Mpp, Mp, w))
                emit(b, jM, jz, jx, jy, f[:, None, None, None] * prod)

        return (np.concatenate(out_r), np.concatenate(out_c), np.concatenate(out_v))

    def rows(self, E, row_index):
        """Sparse rows of A(E) for the given global row indices (any order)."""
        row_index = np.asarray(row_index, dtype=np.int64)
        R, C, V = [], [], []
        for a in range(3):
            for iM in range(self.nM):
                o = self.offsets[a][iM]
                mask = (row_index >= o) & (row_index < o + self.block[a])
                if not np.any(mask):
                    continue
                pos = np.nonzero(mask)[0]
                r, c, v = self._rows(a, iM, row_index[mask] - o, E)
                R.append(pos[r])
                C.append(c)
                V.append(v)
        return sp.csr_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))),
                             shape=(row_index.size, self.N))

    def assemble(self, E):
        """The full N x N matrix A(E) = H - E S (CSR)."""
        return self.rows(E, np.arange(self.N))

    def mass_rows(self, row_index):
        """Rows of S (block diagonal basis-at-points matrix): A(0) - A(1)."""
        return self.rows(0.0, row_index) - self.rows(1.0, row_index)

    # -- separable left-hand block of eq. (FM-fin) ---------------------------
    def separable_block(self, a, E, couple_m=False):
        """L_alpha: the discretised left-hand operator of eq. (FM-fin) for
        component alpha at energy E (Sec. 3.2, the L_{alpha M'M'} blocks).

        With couple_m=False the M'+-1 blocks are dropped (block-Jacobi in M').
        Returns a CSR matrix of size nM * n_z n_x n_y.
        """
        d = self.desc
        J = self.J
        bz, bx, by = self.bz[a], self.bx[a], self.by[a]
        Sz, D1z, D2z = bz.matrix(0), bz.matrix(1), bz.matrix(2)
        Sx, D2x = bx.matrix(0), bx.matrix(2)
        Sy, D2y = by.matrix(0), by.matrix(2)
        z, x, y = bz.points, bx.points, by.points
        Xr2 = np.diag(1.0 / x ** 2)
        Yr2 = np.diag(1.0 / y ** 2)
        Vx = np.diag(ph.coulomb(d["masses"], d["charges"], a, x))
        Vh = np.diag(ph.v_hat(d, a, y))
        K = sp.kron
        blocks = [[None] * self.nM for _ in range(self.nM)]
        for iM, Mp in enumerate(self.Mps):
            Dz = np.diag(1 - z * z) @ D2z - 2 * (Mp + 1) * np.diag(z) @ D1z - Mp * (Mp + 1) * Sz
            L = (-K(Sz, K(Sx, D2y)) - K(Sz, K(D2x, Sy))
                 + (J * (J + 1) - 2 * Mp * Mp) * K(Sz, K(Sx, Yr2 @ Sy))
                 - K(Dz, K(Sx, Yr2 @ Sy)) - K(Dz, K(Xr2 @ Sx, Sy))
                 + K(Sz, K(Vx @ Sx, Sy)) + K(Sz, K(Sx, Vh @ Sy)) - E * K(Sz, K(Sx, Sy)))
            blocks[iM][iM] = L
            if couple_m:
                if iM + 1 < self.nM:
                    Dp = -np.diag(1 - z * z) @ D1z + 2 * (Mp + 1) * np.diag(z) @ Sz
                    blocks[iM][iM + 1] = lam_hat_plus(J, Mp) * K(Dp, K(Sx, Yr2 @ Sy))
                if iM - 1 >= 0:
                    Dm = -D1z
                    blocks[iM][iM - 1] = -lam_hat_minus(J, Mp) * K(Dm, K(Sx, Yr2 @ Sy))
        return sp.bmat(blocks, format="csr")

    def separable(self, E, couple_m=False):
        """Block-diagonal (over alpha) separable operator."""
        return sp.block_diag([self.separable_block(a, E, couple_m) for a in range(3)], format="csr")
