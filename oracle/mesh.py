"""Box meshes, entity numbering and the global DoF map (oracle side).

Domain Omega = [lo, hi] (paper Sec. 2) meshed by n = (n_x, n_y[, n_z]) equal boxes.

Global entity numbering (x fastest everywhere):
 2D  x-edges (i<nx, j<=ny): j*nx+i;  y-edges (i<=nx, j<ny): j*(nx+1)+i;  cells j*nx+i.
 3D  x-edges (i<nx, j<=ny, k<=nz): (k*(ny+1)+j)*nx+i
     y-edges (i<=nx, j<ny, k<=nz): (k*ny+j)*(nx+1)+i
     z-edges (i<=nx, j<=ny, k<nz): (k*(ny+1)+j)*(nx+1)+i
     x-faces (i<=nx, j<ny, k<nz):  (k*ny+j)*(nx+1)+i
     y-faces (i<nx, j<=ny, k<nz):  (k*(ny+1)+j)*nx+i
     z-faces (i<nx, j<ny, k<=nz):  (k*ny+j)*nx+i
     cells: (k*ny+j)*nx+i
Every edge is oriented along +axis and every face frame is (+t1, +t2), so a
shared entity carries the same parametrisation in all cells touching it (cells
are translates): no sign flips.

Global DoF blocks, in order: edge DoFs (by edge family x, y[, z], p+1 per
edge), then [3D] face DoFs (x-, y-, z-faces, 2p(p+1) per face), then cell
interiors (n_interior per cell).  Within an entity the order is the local one of
``oracle.fe``.
"""
import numpy as np

from . import fe


class BoxMesh:
    def __init__(self, dim, n, lo=None, hi=None, p=0):
        self.dim = dim
        self.n = tuple(int(v) for v in n[:dim])
        self.lo = np.zeros(dim) if lo is None else np.asarray(lo[:dim], dtype=np.float64)
        self.hi = np.ones(dim) if hi is None else np.asarray(hi[:dim], dtype=np.float64)
        self.p = p
        self.h = (self.hi - self.lo) / np.asarray(self.n)
        self._number()

    # -- counts -------------------------------------------------------------
    def _number(self):
        d, p = self.dim, self.p
        pe = p + 1
        if d == 2:
            nx, ny = self.n
            self.n_edges = [nx * (ny + 1), (nx + 1) * ny]
            self.n_faces = []
            self.n_cells = nx * ny
        else:
            nx, ny, nz = self.n
            self.n_edges = [nx * (ny + 1) * (nz + 1), (nx + 1) * ny * (nz + 1), (nx + 1) * (ny + 1) * nz]
            self.n_faces = [(nx + 1) * ny * nz, nx * (ny + 1) * nz, nx * ny * (nz + 1)]
            self.n_cells = nx * ny * nz
        self.pf = 2 * p * (p + 1)
        self.pi = fe.n_interior(d, p)
        off = 0
        self.edge_off = []
        for ne in self.n_edges:
            self.edge_off.append(off)
            off += ne * pe
        self.face_off = []
        for nf in self.n_faces:
            self.face_off.append(off)
            off += nf * self.pf
        self.cell_off = off
        off += self.n_cells * self.pi
        self.n_dofs = off
        self.n_loc = fe.n_local(d, p)

    # -- entity ids ---------------------------------------------------------
    def edge_id(self, axis, i, j, k=0):
        if self.dim == 2:
            nx, ny = self.n
            return j * nx + i if axis == 0 else j * (nx + 1) + i
        nx, ny, nz = self.n
        if axis == 0:
            return (k * (ny + 1) + j) * nx + i
        if axis == 1:
            return (k * ny + j) * (nx + 1) + i
        return (k * (ny + 1) + j) * (nx + 1) + i

    def face_id(self, axis, i, j, k):
        nx, ny, nz = self.n
        if axis == 0:
            return (k * ny + j) * (nx + 1) + i
        if axis == 1:
            return (k * (ny + 1) + j) * nx + i
        return (k * ny + j) * nx + i

    def cell_index(self, c):
        if self.dim == 2:
            nx, _ = self.n
            return (c % nx, c // nx)
        nx, ny, _ = self.n
        return (c % nx, (c // nx) % ny, c // (nx * ny))

    def edge_dofs(self, axis, eid):
        pe = self.p + 1
        return self.edge_off[axis] + eid * pe + np.arange(pe)

    def face_dofs(self, axis, fid):
        return self.face_off[axis] + fid * self.pf + np.arange(self.pf)

    # -- cell -> global DoF table ------------------------------------------
    def cell_dofs(self):
        """(n_cells, n_loc) int64 table of global DoFs in local order."""
        d, p = self.dim, self.p
        pe = p + 1
        T = np.zeros((self.n_cells, self.n_loc), dtype=np.int64)
        for c in range(self.n_cells):
            idx = self.cell_index(c)
            row = []
            if d == 2:
                i, j = idx
                row += list(self.edge_dofs(0, self.edge_id(0, i, j)))
                row += list(self.edge_dofs(0, self.edge_id(0, i, j + 1)))
                row += list(self.edge_dofs(1, self.edge_id(1, i, j)))
                row += list(self.edge_dofs(1, self.edge_id(1, i + 1, j)))
            else:
                i, j, k = idx
                for comp in range(3):
                    for jb in (0, 1):
                        for kc in (0, 1):
                            pos = [i, j, k]
                            b, cc = [a for a in range(3) if a != comp]
                            pos[b] += jb
                            pos[cc] += kc
                            row += list(self.edge_dofs(comp, self.edge_id(comp, *pos)))
                for n in range(3):
                    for side in (0, 1):
                        pos = [i, j, k]
                        pos[n] += side
                        row += list(self.face_dofs(n, self.face_id(n, *pos)))
            row += list(self.cell_off + c * self.pi + np.arange(self.pi))
            T[c] = row
        assert T.shape[1] == self.n_loc
        return T

    def cell_origin(self, c):
        return self.lo + np.asarray(self.cell_index(c)) * self.h

    # -- boundary sides -----------------------------------------------------
    def side_cells(self, axis, side):
        """Cells touching the box side {x_axis = lo/hi}, with the local side index."""
        out = []
        for c in range(self.n_cells):
            idx = self.cell_index(c)
            if (side == 0 and idx[axis] == 0) or (side == 1 and idx[axis] == self.n[axis] - 1):
                out.append(c)
        return np.asarray(out, dtype=np.int64)

    def side_dofs(self, axis, side):
        """Global DoFs with nonzero tangential trace on the box side (its closure)."""
        T = self.cell_dofs() if not hasattr(self, "_T") else self._T
        loc = fe.face_functions(self.dim, self.p, axis, side)
        cells = self.side_cells(axis, side)
        return np.unique(T[np.ix_(cells, loc)].ravel())

    def dof_positions2(self):
        """(n_dofs, dim) int64: twice the position, in cells, of the entity carrying each DoF
        (an x-edge (i, j, k) sits at (2i+1, 2j, 2k), an x-face at (2i, 2j+1, 2k+1), a cell at
        (2i+1, 2j+1, 2k+1)).  Used only to order the unknowns of the sparse LU."""
        d, pe, n = self.dim, self.p + 1, self.n

        def grid(shape):  # entity indices, x fastest, as rows (i, j[, k])
            return np.indices(tuple(reversed(shape))).reshape(len(shape), -1)[::-1].T

        X = np.zeros((self.n_dofs, d), dtype=np.int64)
        for a in range(d):
            g = 2 * grid([n[b] + (0 if b == a else 1) for b in range(d)])
            g[:, a] += 1
            X[self.edge_off[a]:self.edge_off[a] + len(g) * pe] = np.repeat(g, pe, axis=0)
        if d == 3:
            for a in range(3):
                g = 2 * grid([n[b] + (1 if b == a else 0) for b in range(3)]) + 1
                g[:, a] -= 1
                X[self.face_off[a]:self.face_off[a] + len(g) * self.pf] = np.repeat(g, self.pf, axis=0)
        g = 2 * grid(list(n)) + 1
        X[self.cell_off:] = np.repeat(g, self.pi, axis=0)
        return X

    def table(self):
        if not hasattr(self, "_T"):
            self._T = self.cell_dofs()
        return self._T


def expected_counts(dim, m, p):
    """Closed-form N for an m^dim mesh (used as a check of the numbering)."""
    if dim == 2:
        return 2 * m * (m + 1) * (p + 1) + 2 * m * m * p * (p + 1)
    return (3 * m * (m + 1) ** 2 * (p + 1) + 3 * (m + 1) * m * m * 2 * p * (p + 1)
            + m ** 3 * 3 * p * p * (p + 1))
