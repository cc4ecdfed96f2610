// Host-side mesh topology: entity/DoF numbering, CSR patterns and gather maps.
//
// Integer bookkeeping only; all arithmetic of the method runs in the HIP kernels.
//
// Numbering (x fastest everywhere), matching the C ABI's documented DoF order:
//  2D  x-edges (i<nx, j<=ny) j*nx+i; y-edges (i<=nx, j<ny) j*(nx+1)+i; cells j*nx+i.
//  3D  x-edges (k*(ny+1)+j)*nx+i, y-edges (k*ny+j)*(nx+1)+i, z-edges (k*(ny+1)+j)*(nx+1)+i,
//      x-faces (k*ny+j)*(nx+1)+i, y-faces (k*(ny+1)+j)*nx+i, z-faces (k*ny+j)*nx+i.
//  DoF blocks: edges (p+1 each) by family, [3D faces (2p(p+1) each)], cell interiors.
// Local shape functions of component a: L_i(t_a) l_jb(t_b) l_kc(t_c), (b<c) the other
// axes; entity = edge if jb,kc in {0,1}, face if exactly one >= 2, interior otherwise.
#include <algorithm>
#include <numeric>

#include "kernels.h"

namespace thm {

static void other_axes(int comp, int &b, int &c) {
    b = comp == 0 ? 1 : 0;
    c = comp == 2 ? 1 : 2;
}

void Topo::build(int dim_, int p_, const int *cells, const double *lo_, const double *hi_) {
    dim = dim_;
    p = p_;
    for (int a = 0; a < 3; ++a) {
        n[a] = a < dim ? cells[a] : 1;
        lo[a] = a < dim ? lo_[a] : 0.0;
        hi[a] = a < dim ? hi_[a] : 1.0;
        h[a] = (hi[a] - lo[a]) / n[a];
    }
    pe = p + 1;
    pf = 2 * p * (p + 1);
    const int64_t nx = n[0], ny = n[1], nz = n[2];
    if (dim == 2) {
        n_edges[0] = nx * (ny + 1);
        n_edges[1] = (nx + 1) * ny;
        n_edges[2] = 0;
        n_cells = nx * ny;
        n_int = 2 * p * (p + 1);
        n_loc = 2 * (p + 1) * (p + 2);
    } else {
        n_edges[0] = nx * (ny + 1) * (nz + 1);
        n_edges[1] = (nx + 1) * ny * (nz + 1);
        n_edges[2] = (nx + 1) * (ny + 1) * nz;
        n_faces[0] = (nx + 1) * ny * nz;
        n_faces[1] = nx * (ny + 1) * nz;
        n_faces[2] = nx * ny * (nz + 1);
        n_cells = nx * ny * nz;
        n_int = 3 * p * p * (p + 1);
        n_loc = 3 * (p + 1) * (p + 2) * (p + 2);
    }
    int64_t off = 0;
    for (int a = 0; a < 3; ++a) { edge_off[a] = off; off += n_edges[a] * pe; }
    for (int a = 0; a < 3; ++a) { face_off[a] = off; off += n_faces[a] * pf; }
    cell_off = off;
    off += n_cells * n_int;
    n_dofs = off;

    // local functions in local order
    fns.clear();
    if (dim == 2) {
        const int es[4][2] = {{0, 0}, {0, 1}, {1, 0}, {1, 1}};
        for (auto &e : es)
            for (int i = 0; i <= p; ++i) fns.push_back({e[0], i, e[1], 0});
        for (int comp = 0; comp < 2; ++comp)
            for (int j = 2; j <= p + 1; ++j)
                for (int i = 0; i <= p; ++i) fns.push_back({comp, i, j, 0});
    } else {
        for (int comp = 0; comp < 3; ++comp)
            for (int jb = 0; jb < 2; ++jb)
                for (int kc = 0; kc < 2; ++kc)
                    for (int i = 0; i <= p; ++i) fns.push_back({comp, i, jb, kc});
        for (int nax = 0; nax < 3; ++nax)
            for (int side = 0; side < 2; ++side)
                for (int comp = 0; comp < 3; ++comp) {
                    if (comp == nax) continue;
                    int b, c;
                    other_axes(comp, b, c);
                    const int m = 3 - nax - comp;  // tangential axis carrying the bubble
                    for (int bub = 2; bub <= p + 1; ++bub)
                        for (int i = 0; i <= p; ++i) {
                            int idx[3] = {0, 0, 0};
                            idx[nax] = side;
                            idx[m] = bub;
                            fns.push_back({comp, i, idx[b], idx[c]});
                        }
                }
        for (int comp = 0; comp < 3; ++comp)
            for (int jb = 2; jb <= p + 1; ++jb)
                for (int kc = 2; kc <= p + 1; ++kc)
                    for (int i = 0; i <= p; ++i) fns.push_back({comp, i, jb, kc});
    }
    if ((int)fns.size() != n_loc) fail(THM_EINVAL, "internal: local function count mismatch");

    for (int s = 0; s < 6; ++s) side_fns[s].clear();
    for (int axis = 0; axis < dim; ++axis)
        for (int side = 0; side < 2; ++side)
            for (int u = 0; u < n_loc; ++u) {
                const LocalFn &f = fns[u];
                if (f.comp == axis) continue;
                int nidx;
                if (dim == 2) {
                    nidx = f.jb;
                } else {
                    int b, c;
                    other_axes(f.comp, b, c);
                    nidx = (axis == b) ? f.jb : f.kc;
                }
                if (nidx == side) side_fns[2 * axis + side].push_back(u);
            }

    // cell -> DoF table
    cell_dofs.assign((size_t)n_cells * n_loc, 0);
    for (int64_t c = 0; c < n_cells; ++c) {
        int ijk[3];
        cell_ijk(c, ijk);
        int32_t *row = &cell_dofs[(size_t)c * n_loc];
        int u = 0;
        if (dim == 2) {
            const int64_t e4[4] = {edge_off[0] + edge_id(0, ijk[0], ijk[1], 0) * pe,
                                   edge_off[0] + edge_id(0, ijk[0], ijk[1] + 1, 0) * pe,
                                   edge_off[1] + edge_id(1, ijk[0], ijk[1], 0) * pe,
                                   edge_off[1] + edge_id(1, ijk[0] + 1, ijk[1], 0) * pe};
            for (int e = 0; e < 4; ++e)
                for (int a = 0; a < pe; ++a) row[u++] = (int32_t)(e4[e] + a);
        } else {
            for (int comp = 0; comp < 3; ++comp) {
                int b, c2;
                other_axes(comp, b, c2);
                for (int jb = 0; jb < 2; ++jb)
                    for (int kc = 0; kc < 2; ++kc) {
                        int pos[3] = {ijk[0], ijk[1], ijk[2]};
                        pos[b] += jb;
                        pos[c2] += kc;
                        const int64_t base = edge_off[comp] + edge_id(comp, pos[0], pos[1], pos[2]) * pe;
                        for (int a = 0; a < pe; ++a) row[u++] = (int32_t)(base + a);
                    }
            }
            for (int nax = 0; nax < 3; ++nax)
                for (int side = 0; side < 2; ++side) {
                    int pos[3] = {ijk[0], ijk[1], ijk[2]};
                    pos[nax] += side;
                    const int64_t base = face_off[nax] + face_id(nax, pos[0], pos[1], pos[2]) * pf;
                    for (int a = 0; a < pf; ++a) row[u++] = (int32_t)(base + a);
                }
        }
        for (int a = 0; a < n_int; ++a) row[u++] = (int32_t)(cell_off + c * n_int + a);
    }
}

int64_t Topo::edge_id(int axis, int i, int j, int k) const {
    const int64_t nx = n[0], ny = n[1];
    if (dim == 2) return axis == 0 ? (int64_t)j * nx + i : (int64_t)j * (nx + 1) + i;
    if (axis == 0) return ((int64_t)k * (ny + 1) + j) * nx + i;
    if (axis == 1) return ((int64_t)k * ny + j) * (nx + 1) + i;
    return ((int64_t)k * (ny + 1) + j) * (nx + 1) + i;
}

int64_t Topo::face_id(int axis, int i, int j, int k) const {
    const int64_t nx = n[0], ny = n[1];
    if (axis == 0) return ((int64_t)k * ny + j) * (nx + 1) + i;
    if (axis == 1) return ((int64_t)k * (ny + 1) + j) * nx + i;
    return ((int64_t)k * ny + j) * nx + i;
}

void Topo::cell_ijk(int64_t c, int *ijk) const {
    ijk[0] = (int)(c % n[0]);
    ijk[1] = (int)((c / n[0]) % n[1]);
    ijk[2] = dim == 3 ? (int)(c / ((int64_t)n[0] * n[1])) : 0;
}

bool Topo::cell_on_side(int64_t c, int axis, int side) const {
    int ijk[3];
    cell_ijk(c, ijk);
    return side == 0 ? ijk[axis] == 0 : ijk[axis] == n[axis] - 1;
}

// Counting sort of (key, value) pairs into CSR form.
static void bucket(int64_t nkeys, const std::vector<int64_t> &key, const std::vector<int32_t> &val,
                   std::vector<int32_t> &ptr, std::vector<int32_t> &out) {
    ptr.assign(nkeys + 1, 0);
    for (int64_t k : key) ptr[k + 1]++;
    for (int64_t i = 0; i < nkeys; ++i) ptr[i + 1] += ptr[i];
    out.assign(val.size(), 0);
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (size_t i = 0; i < key.size(); ++i) out[fill[key[i]]++] = val[i];
}

void build_csr(const Topo &t, HostCSR &K) {
    const int64_t N = t.n_dofs, nc = t.n_cells;
    const int nl = t.n_loc;
    if ((double)nc * nl * nl > 2.0e9) fail(THM_EUNSUPPORTED, "mesh too large for 32-bit element indices");
    // DoF -> cells
    std::vector<int32_t> dc_ptr(N + 1, 0), dc;
    for (int64_t c = 0; c < nc; ++c)
        for (int u = 0; u < nl; ++u) dc_ptr[t.cell_dofs[c * nl + u] + 1]++;
    for (int64_t i = 0; i < N; ++i) dc_ptr[i + 1] += dc_ptr[i];
    dc.assign(dc_ptr[N], 0);
    {
        std::vector<int32_t> fill(dc_ptr.begin(), dc_ptr.end() - 1);
        for (int64_t c = 0; c < nc; ++c)
            for (int u = 0; u < nl; ++u) dc[fill[t.cell_dofs[c * nl + u]]++] = (int32_t)c;
    }
    K.nrows = N;
    K.rowptr.assign(N + 1, 0);
    K.col.clear();
    std::vector<int32_t> tmp;
    for (int64_t r = 0; r < N; ++r) {
        tmp.clear();
        for (int32_t q = dc_ptr[r]; q < dc_ptr[r + 1]; ++q) {
            const int32_t *row = &t.cell_dofs[(size_t)dc[q] * nl];
            tmp.insert(tmp.end(), row, row + nl);
        }
        std::sort(tmp.begin(), tmp.end());
        tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
        K.col.insert(K.col.end(), tmp.begin(), tmp.end());
        K.rowptr[r + 1] = (int32_t)K.col.size();
        if (K.col.size() > (size_t)INT32_MAX) fail(THM_EUNSUPPORTED, "nnz exceeds 32-bit range");
    }
    // gather map: element entry e = c*nl*nl + u*nl + v -> slot
    const int64_t ne = nc * nl * nl;
    std::vector<int64_t> key(ne);
    std::vector<int32_t> val(ne);
    for (int64_t c = 0; c < nc; ++c) {
        const int32_t *row = &t.cell_dofs[(size_t)c * nl];
        for (int u = 0; u < nl; ++u) {
            const int32_t r = row[u];
            const int32_t *b = &K.col[K.rowptr[r]], *e = &K.col[K.rowptr[r + 1]];
            for (int v = 0; v < nl; ++v) {
                const int64_t idx = (c * nl + u) * nl + v;
                key[idx] = K.rowptr[r] + (std::lower_bound(b, e, row[v]) - b);
                val[idx] = (int32_t)idx;
            }
        }
    }
    bucket((int64_t)K.col.size(), key, val, K.gptr, K.gsrc);
}

void build_side_csr(const Topo &t, const std::vector<Side> &sides, HostCSR &C) {
    const int64_t N = t.n_dofs;
    const int nl = t.n_loc;
    const int nf = sides.empty() ? 0 : (int)t.side_fns[0].size();
    std::vector<std::vector<int32_t>> rows(N);
    for (const Side &s : sides) {
        const auto &sf = t.side_fns[2 * s.axis + s.side];
        const int32_t *cd = &t.cell_dofs[(size_t)s.cell * nl];
        for (int a : sf)
            for (int b : sf) rows[cd[a]].push_back(cd[b]);
    }
    C.nrows = N;
    C.rowptr.assign(N + 1, 0);
    C.col.clear();
    for (int64_t r = 0; r < N; ++r) {
        auto &v = rows[r];
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
        C.col.insert(C.col.end(), v.begin(), v.end());
        C.rowptr[r + 1] = (int32_t)C.col.size();
        std::vector<int32_t>().swap(v);
    }
    std::vector<int64_t> key;
    std::vector<int32_t> val;
    for (size_t si = 0; si < sides.size(); ++si) {
        const Side &s = sides[si];
        const auto &sf = t.side_fns[2 * s.axis + s.side];
        const int32_t *cd = &t.cell_dofs[(size_t)s.cell * nl];
        for (int a = 0; a < nf; ++a) {
            const int32_t r = cd[sf[a]];
            const int32_t *b = &C.col[C.rowptr[r]], *e = &C.col[C.rowptr[r + 1]];
            for (int bb = 0; bb < nf; ++bb) {
                key.push_back(C.rowptr[r] + (std::lower_bound(b, e, cd[sf[bb]]) - b));
                val.push_back((int32_t)((si * nf + a) * nf + bb));
            }
        }
    }
    bucket((int64_t)C.col.size(), key, val, C.gptr, C.gsrc);
}

// Layer (stacking index along the last axis) of a skeleton DoF; -1 for interiors.
static int dof_layer(const Topo &t, int64_t g) {
    if (g >= t.cell_off) return -1;
    const int64_t nx = t.n[0], ny = t.n[1];
    if (t.dim == 2) {
        if (g < t.edge_off[1]) return (int)(((g - t.edge_off[0]) / t.pe) / nx);
        return (int)(((g - t.edge_off[1]) / t.pe) / (nx + 1));
    }
    if (g < t.edge_off[1]) return (int)(((g - t.edge_off[0]) / t.pe) / (nx * (ny + 1)));
    if (g < t.edge_off[2]) return (int)(((g - t.edge_off[1]) / t.pe) / ((nx + 1) * ny));
    if (g < t.face_off[0]) return (int)(((g - t.edge_off[2]) / t.pe) / ((nx + 1) * (ny + 1)));
    if (g < t.face_off[1]) return (int)(((g - t.face_off[0]) / t.pf) / ((nx + 1) * ny));
    if (g < t.face_off[2]) return (int)(((g - t.face_off[1]) / t.pf) / (nx * (ny + 1)));
    return (int)(((g - t.face_off[2]) / t.pf) / (nx * ny));
}

void build_layering(const Topo &t, const std::vector<uint8_t> &dir, Layering &L) {
    const int last = t.dim - 1;
    L.nlayers = t.n[last] + 1;
    const int nL = L.nlayers;
    const int64_t N = t.n_dofs;
    L.bsize.assign(nL, 0);
    for (int64_t g = 0; g < t.cell_off; ++g) L.bsize[dof_layer(t, g)]++;
    L.boff.assign(nL + 1, 0);
    for (int k = 0; k < nL; ++k) L.boff[k + 1] = L.boff[k] + L.bsize[k];
    L.n_skel = L.boff[nL];
    L.pboff.assign(nL + 1, 0);
    for (int k = 0; k < nL; ++k)
        L.pboff[k + 1] = L.pboff[k] + (L.bsize[k] + SKEL_ALIGN - 1) / SKEL_ALIGN * SKEL_ALIGN;
    L.n_skel_pad = L.pboff[nL];
    L.skel_pos.assign(L.n_skel, 0);
    for (int k = 0; k < nL; ++k)
        for (int32_t j = 0; j < L.bsize[k]; ++j) L.skel_pos[L.boff[k] + j] = (int32_t)(L.pboff[k] + j);
    L.skel_dof.assign(L.n_skel, 0);
    L.dof_pos.assign(N, -1);
    {
        std::vector<int64_t> fill(L.boff.begin(), L.boff.end() - 1);
        for (int64_t g = 0; g < t.cell_off; ++g) {  // ascending global id within a layer
            const int k = dof_layer(t, g);
            L.skel_dof[fill[k]] = (int32_t)g;
            L.dof_pos[g] = (int32_t)fill[k]++;
        }
    }
    L.sinv_off.assign(nL, 0);
    L.lf_off.assign(nL, -1);
    int64_t so = 0, lo = 0;
    for (int k = 0; k < nL; ++k) {
        L.sinv_off[k] = so;
        so += (int64_t)L.bsize[k] * L.bsize[k];
        if (k > 0) {
            L.lf_off[k] = lo;
            lo += (int64_t)L.bsize[k] * L.bsize[k - 1];
        }
    }
    L.sinv_total = so;
    L.lf_total = lo;

    // condensed element entries -> unique dense targets
    const int nl = t.n_loc, ne = t.n_loc - t.n_int;
    std::vector<std::pair<int64_t, int32_t>> pairs;  // (encoded target, source)
    pairs.reserve((size_t)t.n_cells * ne * ne / 2 + 16);
    for (int64_t c = 0; c < t.n_cells; ++c) {
        const int32_t *cd = &t.cell_dofs[(size_t)c * nl];
        for (int u = 0; u < ne; ++u) {
            const int32_t gu = cd[u];
            if (dir[gu]) continue;
            const int32_t pu = L.dof_pos[gu];
            const int lu = dof_layer(t, gu);
            for (int v = 0; v < ne; ++v) {
                const int32_t gv = cd[v];
                if (dir[gv]) continue;
                const int lv = dof_layer(t, gv);
                const int32_t pv = L.dof_pos[gv];
                int64_t enc;
                if (lu == lv) {
                    enc = 2 * (L.sinv_off[lu] + (int64_t)(pu - L.boff[lu]) * L.bsize[lu] + (pv - L.boff[lv]));
                } else if (lu == lv + 1) {
                    enc = 2 * (L.lf_off[lu] + (int64_t)(pu - L.boff[lu]) * L.bsize[lv] + (pv - L.boff[lv])) + 1;
                } else {
                    continue;
                }
                pairs.push_back({enc, (int32_t)((c * ne + u) * ne + v)});
            }
        }
    }
    std::sort(pairs.begin(), pairs.end());
    L.tgt_index.clear();
    L.tgt_kind.clear();
    L.tgt_ptr.assign(1, 0);
    L.tgt_src.clear();
    for (size_t i = 0; i < pairs.size(); ++i) {
        if (i == 0 || pairs[i].first != pairs[i - 1].first) {
            if (i) L.tgt_ptr.push_back((int32_t)L.tgt_src.size());
            L.tgt_index.push_back(pairs[i].first >> 1);
            L.tgt_kind.push_back((int32_t)(pairs[i].first & 1));
        }
        L.tgt_src.push_back(pairs[i].second);
    }
    L.tgt_ptr.push_back((int32_t)L.tgt_src.size());

    // skeleton position -> (cell, local skeleton index)
    std::vector<int64_t> key;
    std::vector<int32_t> valc, vall;
    for (int64_t c = 0; c < t.n_cells; ++c) {
        const int32_t *cd = &t.cell_dofs[(size_t)c * nl];
        for (int u = 0; u < ne; ++u) {
            key.push_back(L.dof_pos[cd[u]]);
            valc.push_back((int32_t)c);
            vall.push_back(u);
        }
    }
    std::vector<int32_t> ptr2;
    bucket(L.n_skel, key, valc, L.cond_ptr, L.cond_cell);
    bucket(L.n_skel, key, vall, ptr2, L.cond_loc);
}

}  // namespace thm

namespace thm {
// SELL-64 layout of a CSR pattern (see MatDesc).  Rows are sorted by decreasing length
// inside windows of SELL_SIGMA consecutive rows (stable, so equal lengths keep their
// order), then cut into slices of 64; row[s * 64 + lane] is the original row of a lane
// (-1 past the last row).  Entry (k, lane) of slice s sits at ptr[s] + 64 k + lane; rows
// shorter than the slice's longest row are padded with src = -1 and a valid column.
void sell_build(int64_t n, const std::vector<int32_t> &rowptr, const std::vector<int32_t> &col,
                std::vector<int32_t> &ptr, std::vector<int32_t> &scol, std::vector<int32_t> &src,
                std::vector<int32_t> &row) {
    const int64_t nsl = (n + SELL_C - 1) / SELL_C;
    row.assign(nsl * SELL_C, -1);
    for (int64_t w0 = 0; w0 < n; w0 += SELL_SIGMA) {
        const int64_t w1 = std::min<int64_t>(n, w0 + SELL_SIGMA);
        std::vector<int32_t> ord(w1 - w0);
        std::iota(ord.begin(), ord.end(), (int32_t)w0);
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
            return rowptr[a + 1] - rowptr[a] > rowptr[b + 1] - rowptr[b];
        });
        std::copy(ord.begin(), ord.end(), row.begin() + w0);
    }
    auto len = [&](int64_t slot) { return row[slot] < 0 ? 0 : rowptr[row[slot] + 1] - rowptr[row[slot]]; };
    ptr.assign(nsl + 1, 0);
    int64_t tot = 0;
    for (int64_t s = 0; s < nsl; ++s) {
        int32_t w = 0;
        for (int lane = 0; lane < SELL_C; ++lane) w = std::max(w, len(s * SELL_C + lane));
        tot += (int64_t)w * SELL_C;
        if (tot > INT32_MAX) fail(THM_EUNSUPPORTED, "matrix too large for 32-bit SELL offsets");
        ptr[s + 1] = (int32_t)tot;
    }
    scol.assign(tot, 0);
    src.assign(tot, -1);
    for (int64_t s = 0; s < nsl; ++s) {
        const int32_t w = (ptr[s + 1] - ptr[s]) / SELL_C;
        for (int lane = 0; lane < SELL_C; ++lane) {
            const int32_t r = row[s * SELL_C + lane];
            const int32_t l = len(s * SELL_C + lane);
            for (int32_t k = 0; k < w; ++k) {
                const int64_t e = ptr[s] + (int64_t)k * SELL_C + lane;
                if (k < l) {
                    scol[e] = col[rowptr[r] + k];
                    src[e] = rowptr[r] + k;
                } else {
                    scol[e] = r >= 0 ? r : 0;
                }
            }
        }
    }
}
}  // namespace thm
