// Finite-element kernels for gfx950: reference Nedelec basis tables, batched
// element matrices (eq. (3)), deterministic CSR gathers, boundary trace masses
// (impedance matrix C and the Gamma^inc mass), the incident-field load of the
// Dirichlet projection, lifting helpers, and the adjoint objective/gradient.
//
// Basis (Sec. 2, first-kind tensor-product Nedelec, degree p): component a of a
// local function is L_i(t_a) l_jb(t_b) l_kc(t_c) with (b < c) the other axes,
// L_i(t) = P_i(2t-1) and l_0 = 1-t, l_1 = t, l_j = int_0^t P_{j-1}(2s-1) ds.
// Covariant Piola map on box cells: component a / h_a; curl = J curl_hat / det J.
#include "kernels.h"

namespace thm {

__device__ __forceinline__ void d_legendre(int n, double u, double *P) {
    P[0] = 1.0;
    if (n >= 1) P[1] = u;
    for (int k = 1; k < n; ++k) P[k + 1] = ((2 * k + 1) * u * P[k] - k * P[k - 1]) / (k + 1);
}

// L_i(t)
__device__ __forceinline__ double d_L(int i, double t) {
    double P[12];
    d_legendre(i, 2.0 * t - 1.0, P);
    return P[i];
}

// l_j(t) and l_j'(t)
__device__ __forceinline__ void d_l(int j, double t, double &v, double &d) {
    if (j == 0) { v = 1.0 - t; d = -1.0; return; }
    if (j == 1) { v = t; d = 1.0; return; }
    double P[12];
    d_legendre(j, 2.0 * t - 1.0, P);
    v = (P[j] - P[j - 2]) / (2.0 * (2 * j - 1));
    d = P[j - 1];
}

__device__ __forceinline__ double d_eps(int i, int j, int k) { return 0.5 * (i - j) * (j - k) * (k - i); }

// Reference value (3 comps) and reference curl (1 comp in 2D, 3 in 3D) of local function f at t.
__device__ void d_eval(int dim, const LocalFn f, const double *t, double *val, double *curl) {
    val[0] = val[1] = val[2] = 0.0;
    curl[0] = curl[1] = curl[2] = 0.0;
    const double Li = d_L(f.i, t[f.comp]);
    if (dim == 2) {
        const int o = 1 - f.comp;
        double v, d;
        d_l(f.jb, t[o], v, d);
        val[f.comp] = Li * v;
        curl[0] = (f.comp == 1 ? 1.0 : -1.0) * Li * d;  // d_xi f_y - d_eta f_x
        return;
    }
    const int b = f.comp == 0 ? 1 : 0;
    const int c = f.comp == 2 ? 1 : 2;
    double vb, db, vc, dc;
    d_l(f.jb, t[b], vb, db);
    d_l(f.kc, t[c], vc, dc);
    val[f.comp] = Li * vb * vc;
    const double dfb = Li * db * vc, dfc = Li * vb * dc;
    const int rb = 3 - b - f.comp, rc = 3 - c - f.comp;
    curl[rb] += d_eps(rb, b, f.comp) * dfb;
    curl[rc] += d_eps(rc, c, f.comp) * dfc;
}

// Gauss-Legendre nodes/weights on [0,1] by Newton iteration on P_q.
__global__ void k_gauss(int q, double *x, double *w) {
    const int i = threadIdx.x;
    if (i >= q) return;
    double z = cos(M_PI * (i + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;
        for (int k = 1; k < q; ++k) {
            const double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1);
            p0 = p1;
            p1 = p2;
        }
        const double pq = q == 0 ? 1.0 : (q == 1 ? z : p1);
        const double pqm1 = q == 1 ? 1.0 : p0;
        dp = q * (z * pq - pqm1) / (z * z - 1.0);
        const double dz = pq / dp;
        z -= dz;
        if (fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged node
    {
        double p0 = 1.0, p1 = z;
        for (int k = 1; k < q; ++k) {
            const double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1);
            p0 = p1;
            p1 = p2;
        }
        const double pq = q == 1 ? z : p1;
        const double pqm1 = q == 1 ? 1.0 : p0;
        dp = q * (z * pq - pqm1) / (z * z - 1.0);
    }
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2/((1-z^2)P'^2) scaled by 1/2
}

void fe_gauss(int q, DBuf<double> &x, DBuf<double> &w, hipStream_t st) {
    x.alloc(q);
    w.alloc(q);
    k_gauss<<<1, 64, 0, st>>>(q, x.p, w.p);
    THM_HIP(hipGetLastError());
}

// Tensor points: ndim_pts free axes; fixed axis `axis` (or -1) at value `side`.
__global__ void k_points(int dim, int q, int axis, int side, int base, const double *gx, const double *gw,
                         double *pts, double *w) {
    const int nfree = axis < 0 ? dim : dim - 1;
    int total = 1;
    for (int a = 0; a < nfree; ++a) total *= q;
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= total) return;
    double t[3] = {0, 0, 0};
    double ww = 1.0;
    int r = id;
    for (int a = 0; a < dim; ++a) {
        if (a == axis) { t[a] = side; continue; }
        const int k = r % q;
        r /= q;
        t[a] = gx[k];
        ww *= gw[k];
    }
    for (int a = 0; a < 3; ++a) pts[(int64_t)(base + id) * 3 + a] = t[a];
    w[base + id] = ww;
}

__global__ void k_tables(int dim, int n_loc, int npts, const LocalFn *fns, const double *pts, double *val,
                         double *curl) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)n_loc * npts) return;
    const int u = (int)(id / npts), q = (int)(id % npts);
    double v[3], c[3];
    d_eval(dim, fns[u], pts + (int64_t)q * 3, v, c);
    for (int a = 0; a < 3; ++a) {
        val[((int64_t)u * 3 + a) * npts + q] = v[a];
        curl[((int64_t)u * 3 + a) * npts + q] = c[a];
    }
}

static void build_tables(int dim, int n_loc, const LocalFn *fns, FeTables &T, hipStream_t st) {
    T.val.alloc((size_t)n_loc * 3 * T.npts);
    T.curl.alloc((size_t)n_loc * 3 * T.npts);
    const int64_t tot = (int64_t)n_loc * T.npts;
    k_tables<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(dim, n_loc, T.npts, fns, T.pts.p, T.val.p, T.curl.p);
    THM_HIP(hipGetLastError());
}

void fe_tables_cell(int dim, int p, int q, const LocalFn *fns, int n_loc, FeTables &T, hipStream_t st) {
    (void)p;
    DBuf<double> gx, gw;
    fe_gauss(q, gx, gw, st);
    T.npts = dim == 2 ? q * q : q * q * q;
    T.pts.alloc((size_t)T.npts * 3);
    T.w.alloc(T.npts);
    k_points<<<(T.npts + 255) / 256, 256, 0, st>>>(dim, q, -1, 0, 0, gx.p, gw.p, T.pts.p, T.w.p);
    THM_HIP(hipGetLastError());
    build_tables(dim, n_loc, fns, T, st);
    THM_HIP(hipStreamSynchronize(st));
}

// All 2*dim sides in one table: side st = 2*axis+side owns points [st*nps, (st+1)*nps).
void fe_tables_side(int dim, int p, int q, int, int, const LocalFn *fns, int n_loc, FeTables &T, hipStream_t st) {
    (void)p;
    DBuf<double> gx, gw;
    fe_gauss(q, gx, gw, st);
    const int nps = dim == 2 ? q : q * q;
    T.npts = 2 * dim * nps;
    T.pts.alloc((size_t)T.npts * 3);
    T.w.alloc(T.npts);
    for (int axis = 0; axis < dim; ++axis)
        for (int side = 0; side < 2; ++side)
            k_points<<<(nps + 255) / 256, 256, 0, st>>>(dim, q, axis, side, (2 * axis + side) * nps, gx.p, gw.p,
                                                        T.pts.p, T.w.p);
    THM_HIP(hipGetLastError());
    build_tables(dim, n_loc, fns, T, st);
    THM_HIP(hipStreamSynchronize(st));
}

// Reference matrices of the cell: RM[u][v] = sum_r cm_r sum_q w_q f_u^r f_v^r over the value
// components and RA[u][v] = sum_r cc_r sum_q w_q (curl f_u)^r (curl f_v)^r over the curl
// components, where cm_r, cc_r are the covariant-Piola factors of the cell's edge lengths h.
// On an axis-aligned box that map is diagonal, so every element matrix of eq. (3) is
// K_c = RA / mu_c - w^2 RM (the same sums, in the same order, for every cell).
__global__ void __launch_bounds__(256) k_ref_matrices(int dim, int n_loc, int npts, const double *__restrict__ val,
                                                      const double *__restrict__ curl, const double *__restrict__ w,
                                                      const double *__restrict__ h, double *__restrict__ R) {
    const int64_t nl2 = (int64_t)n_loc * n_loc;
    const int64_t uv = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (uv >= nl2) return;
    const int u = (int)(uv / n_loc), v = (int)(uv % n_loc);
    const double hx = h[0], hy = h[1], hz = dim == 3 ? h[2] : 1.0;
    const double det = hx * hy * hz;
    const double hh[3] = {hx, hy, hz};
    double cm[3], cc[3];
    for (int a = 0; a < 3; ++a) {
        cm[a] = det / (hh[a] * hh[a]);
        cc[a] = dim == 2 ? 1.0 / det : hh[a] * hh[a] / det;
    }
    const int ncomp = dim, ncurl = dim == 2 ? 1 : 3;
    double m = 0.0, a = 0.0;
    for (int r = 0; r < ncomp; ++r) {
        const double *vu = val + ((int64_t)u * 3 + r) * npts, *vv = val + ((int64_t)v * 3 + r) * npts;
        double s = 0.0;
        for (int q = 0; q < npts; ++q) s += w[q] * vu[q] * vv[q];
        m += cm[r] * s;
    }
    for (int r = 0; r < ncurl; ++r) {
        const double *cu = curl + ((int64_t)u * 3 + r) * npts, *cv = curl + ((int64_t)v * 3 + r) * npts;
        double s = 0.0;
        for (int q = 0; q < npts; ++q) s += w[q] * cu[q] * cv[q];
        a += cc[r] * s;
    }
    R[uv] = m;
    R[nl2 + uv] = a;
}

// K_c[u][v] = mu_c^{-1} int curl phi_u . curl phi_v - w^2 int phi_u . phi_v   (eq. (3), K = A - w^2 M):
// one pass over the output.  Block (x, y) owns entries [1024 x, 1024 x + 1024) of the
// element matrix (four per thread, consecutive threads at consecutive addresses) and the
// cells y, y + gridDim.y, ...; the reference entries stay in registers across its cells.
__global__ void __launch_bounds__(256) k_element(int64_t ncells, int n_loc, const double *__restrict__ R,
                                                 const double *__restrict__ mu, const double *__restrict__ eps,
                                                 double omega, double *__restrict__ Kel) {
    const int nl2 = n_loc * n_loc;
    double rm[4], ra[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int uv = blockIdx.x * 1024 + k * 256 + threadIdx.x;
        rm[k] = uv < nl2 ? R[uv] : 0.0;
        ra[k] = uv < nl2 ? R[nl2 + uv] : 0.0;
    }
    const double w2 = omega * omega;
    for (int64_t c = blockIdx.y; c < ncells; c += gridDim.y) {
        const double inv = mu ? 1.0 / mu[c] : 1.0;
        const double we = eps ? w2 * eps[c] : w2;  // relative permittivity weights the mass
        double *K = Kel + c * nl2;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int uv = blockIdx.x * 1024 + k * 256 + threadIdx.x;
            if (uv < nl2) K[uv] = ra[k] * inv - we * rm[k];
        }
    }
}

void launch_element_matrices(int dim, int64_t ncells, int n_loc, FeTables &T, const double *h,
                             const double *mu, const double *eps, double omega, double *Kel, hipStream_t st) {
    const int64_t nl2 = (int64_t)n_loc * n_loc;
    if ((int64_t)T.ref.n != 2 * nl2) {
        T.ref.alloc(2 * nl2);
        k_ref_matrices<<<(unsigned)((nl2 + 255) / 256), 256, 0, st>>>(dim, n_loc, T.npts, T.val.p, T.curl.p, T.w.p, h,
                                                                      T.ref.p);
    }
    if (ncells > 0) {
        const dim3 grid((unsigned)((nl2 + 1023) / 1024), (unsigned)std::min<int64_t>(ncells, 2048));
        k_element<<<grid, 256, 0, st>>>(ncells, n_loc, T.ref.p, mu, eps, omega, Kel);
    }
    THM_HIP(hipGetLastError());
}

__global__ void k_gather(int64_t nnz, const int32_t *__restrict__ gptr, const int32_t *__restrict__ gsrc,
                         const double *__restrict__ src, double scale, double *__restrict__ val) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nnz) return;
    double acc = 0.0;
    for (int32_t e = gptr[s]; e < gptr[s + 1]; ++e) acc += src[gsrc[e]];
    val[s] = scale * acc;
}

void launch_gather(int64_t nnz, const int32_t *gptr, const int32_t *gsrc, const double *src, double scale,
                   double *val, hipStream_t st) {
    if (!nnz) return;
    k_gather<<<(unsigned)((nnz + 255) / 256), 256, 0, st>>>(nnz, gptr, gsrc, src, scale, val);
    THM_HIP(hipGetLastError());
}

// Tangential trace mass on one side entry: int_side gamma^T phi_a . gamma^T phi_b ds.
__global__ void k_side_mass(int dim, int nsides, const int32_t *side_axis, const int32_t *side_side,
                            const int32_t *side_fn, int nf, int n_loc, int nps, const double *val, const double *w,
                            const double *h, double *out) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)nsides * nf * nf) return;
    const int si = (int)(id / (nf * nf));
    const int a = (int)((id / nf) % nf), b = (int)(id % nf);
    const int axis = side_axis[si], sd = side_side[si], stt = 2 * axis + sd;
    const int ua = side_fn[stt * nf + a], ub = side_fn[stt * nf + b];
    const int npts = 2 * dim * nps;
    double ds = 1.0;
    for (int t = 0; t < dim; ++t)
        if (t != axis) ds *= h[t];
    double acc = 0.0;
    for (int t = 0; t < dim; ++t) {
        if (t == axis) continue;
        const double *va = val + ((int64_t)ua * 3 + t) * npts + stt * nps;
        const double *vb = val + ((int64_t)ub * 3 + t) * npts + stt * nps;
        double s = 0.0;
        for (int q = 0; q < nps; ++q) s += w[stt * nps + q] * va[q] * vb[q];
        acc += s / (h[t] * h[t]);
    }
    out[id] = acc * ds;
}

void launch_side_mass(int dim, int nsides, const int32_t *side_axis, const int32_t *side_side,
                      const int32_t *side_fn, int nf, int n_loc, const FeTables *tabs[6], const double *h,
                      double *out, hipStream_t st) {
    if (!nsides) return;
    const FeTables &T = *tabs[0];
    const int nps = T.npts / (2 * dim);
    const int64_t tot = (int64_t)nsides * nf * nf;
    k_side_mass<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(dim, nsides, side_axis, side_side, side_fn, nf,
                                                               n_loc, nps, T.val.p, T.w.p, h, out);
    THM_HIP(hipGetLastError());
}

// out[si] = f in[si] for the side blocks (nf x nf each) whose (axis, side) bit 2 axis + side is
// set in sel, out[si] = in[si] for the others.
__global__ void k_side_scale(int nsides, const int32_t *__restrict__ side_axis, const int32_t *__restrict__ side_side,
                             uint32_t sel, int nf, double f, const double *__restrict__ in, double *__restrict__ out) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)nsides * nf * nf) return;
    const int si = (int)(id / (nf * nf));
    const bool on = (sel >> (2 * side_axis[si] + side_side[si])) & 1u;
    out[id] = on ? f * in[id] : in[id];
}

void launch_side_scale(int nsides, const int32_t *side_axis, const int32_t *side_side, uint32_t sel, int nf,
                       double f, const double *in, double *out, hipStream_t st) {
    const int64_t tot = (int64_t)nsides * nf * nf;
    if (!tot) return;
    k_side_scale<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(nsides, side_axis, side_side, sel, nf, f, in, out);
    THM_HIP(hipGetLastError());
}

// kel[c][u_a][u_b] += coef blk[si][a][b] for the sides si in [s0, s1) of one (axis, side) group, c
// the side's cell and u the side's local functions (a group holds each cell once, so the adds
// of one launch do not collide and every entry is summed in launch order).
__global__ void k_side_to_elem(int s0, int s1, const int32_t *__restrict__ side_cell,
                               const int32_t *__restrict__ side_axis, const int32_t *__restrict__ side_side,
                               const int32_t *__restrict__ side_fn, int nf, int n_loc, double coef,
                               const double *__restrict__ blk, double *__restrict__ kel) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)(s1 - s0) * nf * nf) return;
    const int si = s0 + (int)(id / (nf * nf));
    const int a = (int)((id / nf) % nf), b = (int)(id % nf);
    const int stt = 2 * side_axis[si] + side_side[si];
    const int ua = side_fn[stt * nf + a], ub = side_fn[stt * nf + b];
    kel[((int64_t)side_cell[si] * n_loc + ua) * n_loc + ub] += coef * blk[(int64_t)si * nf * nf + a * nf + b];
}

void launch_side_to_elem(int s0, int s1, const int32_t *side_cell, const int32_t *side_axis,
                         const int32_t *side_side, const int32_t *side_fn, int nf, int n_loc, double coef,
                         const double *blk, double *kel, hipStream_t st) {
    const int64_t tot = (int64_t)(s1 - s0) * nf * nf;
    if (tot <= 0) return;
    k_side_to_elem<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(s0, s1, side_cell, side_axis, side_side, side_fn,
                                                                  nf, n_loc, coef, blk, kel);
    THM_HIP(hipGetLastError());
}

// s_a = int_side gamma^T(E^inc) . gamma^T(phi_a) ds with E^inc = pol exp(-i w d.x); complex output.
__global__ void k_side_load(int dim, int nsides, const int32_t *side_cell, const int32_t *side_axis,
                            const int32_t *side_side, const int32_t *side_fn, int nf, int n_loc, int nps,
                            const double *pts, const double *val, const double *w, const double *h,
                            const double *lo, const int32_t *ncell, const double *dirv, const double *pol_re,
                            const double *pol_im, double omega, double *out) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)nsides * nf) return;
    const int si = (int)(id / nf), a = (int)(id % nf);
    const int axis = side_axis[si], sd = side_side[si], stt = 2 * axis + sd;
    const int ua = side_fn[stt * nf + a];
    const int npts = 2 * dim * nps;
    const int64_t c = side_cell[si];
    int ijk[3];
    ijk[0] = (int)(c % ncell[0]);
    ijk[1] = (int)((c / ncell[0]) % ncell[1]);
    ijk[2] = dim == 3 ? (int)(c / ((int64_t)ncell[0] * ncell[1])) : 0;
    double ds = 1.0;
    for (int t = 0; t < dim; ++t)
        if (t != axis) ds *= h[t];
    double re = 0.0, im = 0.0;
    for (int q = 0; q < nps; ++q) {
        const int qq = stt * nps + q;
        double phase = 0.0;
        for (int t = 0; t < dim; ++t) phase += dirv[t] * (lo[t] + (ijk[t] + pts[(int64_t)qq * 3 + t]) * h[t]);
        double sn, cs;
        sincos(-omega * phase, &sn, &cs);
        double pr = 0.0, pi = 0.0;
        for (int t = 0; t < dim; ++t) {
            if (t == axis) continue;
            const double phi = val[((int64_t)ua * 3 + t) * npts + qq] / h[t];
            pr += pol_re[t] * phi;
            pi += pol_im[t] * phi;
        }
        // (pr + i pi) (cs + i sn)
        re += w[qq] * (pr * cs - pi * sn);
        im += w[qq] * (pr * sn + pi * cs);
    }
    out[2 * id] = re * ds;
    out[2 * id + 1] = im * ds;
}

void launch_side_load(int dim, int nsides, const int32_t *side_cell, const int32_t *side_axis,
                      const int32_t *side_side, const int32_t *side_fn, int nf, int n_loc, const FeTables *tabs[6],
                      const double *h, const double *lo, const int32_t *ncell3, const double *dirv,
                      const double *pol_re, const double *pol_im, double omega, double *out, hipStream_t st) {
    if (!nsides) return;
    const FeTables &T = *tabs[0];
    const int nps = T.npts / (2 * dim);
    const int64_t tot = (int64_t)nsides * nf;
    k_side_load<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(dim, nsides, side_cell, side_axis, side_side,
                                                               side_fn, nf, n_loc, nps, T.pts.p, T.val.p, T.w.p, h,
                                                               lo, ncell3, dirv, pol_re, pol_im, omega, out);
    THM_HIP(hipGetLastError());
}

// out[i] (complex) = sum over e in [ptr[i], ptr[i+1]) of vals[src[e]] (complex)
__global__ void k_gather_vec(int64_t n, const int32_t *ptr, const int32_t *src, const double *vals, double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double re = 0.0, im = 0.0;
    for (int32_t e = ptr[i]; e < ptr[i + 1]; ++e) {
        re += vals[2 * (int64_t)src[e]];
        im += vals[2 * (int64_t)src[e] + 1];
    }
    out[2 * i] = re;
    out[2 * i + 1] = im;
}

void launch_gather_vec(int64_t n, const int32_t *ptr, const int32_t *src, const double *vals, double *out,
                       hipStream_t st) {
    if (!n) return;
    k_gather_vec<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, ptr, src, vals, out);
    THM_HIP(hipGetLastError());
}

// Dirichlet rows/columns -> identity (diag_one) or zero.
__global__ void k_dirichletize(int64_t n, const int32_t *rowptr, const int32_t *col, const uint8_t *dir,
                               double *val, int diag_one) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const bool dr = dir[r];
    for (int32_t q = rowptr[r]; q < rowptr[r + 1]; ++q) {
        const int32_t c = col[q];
        if (dr || dir[c]) val[q] = (diag_one && dr && c == r) ? 1.0 : 0.0;
    }
}

void launch_dirichletize(int64_t n, const int32_t *rowptr, const int32_t *col, const uint8_t *dir, double *val,
                         int diag_one, hipStream_t st) {
    k_dirichletize<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, rowptr, col, dir, val, diag_one);
    THM_HIP(hipGetLastError());
}

// y <- -y on free rows, 0 on Dirichlet rows (complex interleaved).
__global__ void k_lift_finish(int64_t n, const uint8_t *dir, double *y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (dir[i]) { y[2 * i] = 0.0; y[2 * i + 1] = 0.0; }
    else { y[2 * i] = -y[2 * i]; y[2 * i + 1] = -y[2 * i + 1]; }
}

void launch_lift_finish(int64_t n, const uint8_t *dir, double *y, hipStream_t st) {
    k_lift_finish<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, dir, y);
    THM_HIP(hipGetLastError());
}

// x[i] += gD[i] on Dirichlet rows (gD stored full length, complex)
__global__ void k_expand_dir(int64_t n, const uint8_t *dir, const double *g, double *x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !dir[i]) return;
    x[2 * i] = g[2 * i];
    x[2 * i + 1] = g[2 * i + 1];
}

void launch_expand_dirichlet(int64_t n, const uint8_t *dir, const double *gvals, double *x, hipStream_t st) {
    k_expand_dir<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, dir, gvals, x);
    THM_HIP(hipGetLastError());
}

__global__ void k_diag(int64_t n, const int32_t *rowptr, const int32_t *col, const double *val, double *d) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double v = 0.0;
    for (int32_t q = rowptr[r]; q < rowptr[r + 1]; ++q)
        if (col[q] == r) v = val[q];
    d[r] = v;
}

void launch_diag_extract(int64_t n, const int32_t *rowptr, const int32_t *col, const double *val, double *d,
                         hipStream_t st) {
    k_diag<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, rowptr, col, val, d);
    THM_HIP(hipGetLastError());
}

// Per cell: r_c = M_T,c E_c (complex) over cell n T with Gauss q = p+2 on the clipped
// box, and J_c = Re(E_c^H M_T,c E_c).  One block per cell.
__global__ void __launch_bounds__(256) k_target(int dim, int p, int64_t ncells, int n_loc, const LocalFn *fns,
                                                const int32_t *cell_dofs, const double *h, const double *lo,
                                                const int32_t *ncell, const double *tlo, const double *thi,
                                                const double *E, const uint8_t *dir, double *rhs, double *Jc) {
    __shared__ double Er[64], Ei[64];
    __shared__ double Vq[64 * 3 * 8];  // values at the current batch of points (<= 8 points)
    __shared__ double wq[8];
    __shared__ double gx[12], gw[12];
    __shared__ double red[4];
    const int64_t c = blockIdx.x;
    if (c >= ncells) return;
    int ijk[3];
    ijk[0] = (int)(c % ncell[0]);
    ijk[1] = (int)((c / ncell[0]) % ncell[1]);
    ijk[2] = dim == 3 ? (int)(c / ((int64_t)ncell[0] * ncell[1])) : 0;
    double ta[3] = {0, 0, 0}, tb[3] = {1, 1, 1};
    bool empty = false;
    for (int a = 0; a < dim; ++a) {
        const double o = lo[a] + ijk[a] * h[a];
        const double l = fmax(tlo[a], o), r = fmin(thi[a], o + h[a]);
        if (!(r > l)) empty = true;
        ta[a] = (l - o) / h[a];
        tb[a] = (r - o) / h[a];
    }
    const int tid = threadIdx.x;
    if (empty) {
        for (int u = tid; u < n_loc; u += blockDim.x) {
            rhs[((int64_t)c * n_loc + u) * 2] = 0.0;
            rhs[((int64_t)c * n_loc + u) * 2 + 1] = 0.0;
        }
        if (tid == 0) Jc[c] = 0.0;
        return;
    }
    const int q = p + 2;
    if (tid < q) {
        // Gauss nodes (same Newton iteration as k_gauss)
        double z = cos(M_PI * (tid + 0.75) / (q + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 1; k < q; ++k) { const double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1); p0 = p1; p1 = p2; }
            dp = q * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 1; k < q; ++k) { const double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1); p0 = p1; p1 = p2; }
        dp = q * (z * p1 - p0) / (z * z - 1.0);
        gx[tid] = 0.5 * (1.0 - z);
        gw[tid] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
    for (int u = tid; u < n_loc; u += blockDim.x) {
        const int32_t g = cell_dofs[c * n_loc + u];
        Er[u] = E[2 * (int64_t)g];
        Ei[u] = E[2 * (int64_t)g + 1];
    }
    __syncthreads();
    const int npts = dim == 2 ? q * q : q * q * q;
    double det = 1.0, clipw = 1.0;
    for (int a = 0; a < dim; ++a) { det *= h[a]; clipw *= (tb[a] - ta[a]); }
    // accumulate r_u = sum_q w_q phi_u(q) . E_h(q) in registers of thread u
    double rr = 0.0, ri = 0.0, jac = 0.0;
    for (int q0 = 0; q0 < npts; q0 += 8) {
        const int nb = min(8, npts - q0);
        __syncthreads();
        for (int id = tid; id < nb * n_loc; id += blockDim.x) {
            const int k = id / n_loc, u = id % n_loc;
            int r = q0 + k;
            double t[3] = {0, 0, 0};
            double ww = 1.0;
            for (int a = 0; a < dim; ++a) {
                const int kk = r % q;
                r /= q;
                t[a] = ta[a] + (tb[a] - ta[a]) * gx[kk];
                ww *= gw[kk];
            }
            double v[3], cu[3];
            d_eval(dim, fns[u], t, v, cu);
            for (int a = 0; a < 3; ++a) Vq[(k * 64 + u) * 3 + a] = a < dim ? v[a] / h[a] : 0.0;
            if (u == 0) wq[k] = ww * clipw * det;
        }
        __syncthreads();
        if (tid < n_loc) {
            for (int k = 0; k < nb; ++k) {
                double er[3] = {0, 0, 0}, ei[3] = {0, 0, 0};
                for (int v = 0; v < n_loc; ++v)
                    for (int a = 0; a < dim; ++a) {
                        er[a] += Er[v] * Vq[(k * 64 + v) * 3 + a];
                        ei[a] += Ei[v] * Vq[(k * 64 + v) * 3 + a];
                    }
                double dr = 0.0, di = 0.0;
                for (int a = 0; a < dim; ++a) {
                    dr += Vq[(k * 64 + tid) * 3 + a] * er[a];
                    di += Vq[(k * 64 + tid) * 3 + a] * ei[a];
                }
                rr += wq[k] * dr;
                ri += wq[k] * di;
            }
        }
    }
    if (tid < n_loc) {
        rhs[((int64_t)c * n_loc + tid) * 2] = rr;
        rhs[((int64_t)c * n_loc + tid) * 2 + 1] = ri;
        jac = Er[tid] * rr + Ei[tid] * ri;  // Re(conj(E_u) r_u)
    }
    // block reduce J
    double v = jac;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) Jc[c] = red[0] + red[1] + red[2] + red[3];
    (void)dir;
}

void launch_target_rhs(int dim, int p, int64_t ncells, int n_loc, const LocalFn *fns, const int32_t *cell_dofs,
                       const double *h, const double *lo, const int32_t *ncell3, const double *tlo,
                       const double *thi, const double *E, const uint8_t *dir, double *rhs_cells, double *Jcells,
                       hipStream_t st) {
    if (n_loc > 64) fail(THM_EUNSUPPORTED, "adjoint target mass supports at most 64 local DoFs");
    k_target<<<(unsigned)ncells, 256, 0, st>>>(dim, p, ncells, n_loc, fns, cell_dofs, h, lo, ncell3, tlo, thi, E,
                                              dir, rhs_cells, Jcells);
    THM_HIP(hipGetLastError());
}

// dJ/dmu_c = 2 mu_c^{-2} Re(lambda_c^H Ahat_c E_c) = 2 mu_c^{-2} Re int conj(curl lambda) . curl E (unit coefficient)
__global__ void k_cell_grad(int dim, int64_t ncells, int n_loc, int npts, const double *val, const double *curl,
                            const double *w, const int32_t *cell_dofs, const double *h, const double *mu,
                            const double *E, const double *lam, double *grad) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    (void)val;
    const double hh[3] = {h[0], h[1], dim == 3 ? h[2] : 1.0};
    const double det = hh[0] * hh[1] * hh[2];
    const int ncurl = dim == 2 ? 1 : 3;
    double acc = 0.0;
    for (int q = 0; q < npts; ++q) {
        for (int r = 0; r < ncurl; ++r) {
            double er = 0, ei = 0, lr = 0, li = 0;
            for (int u = 0; u < n_loc; ++u) {
                const int32_t g = cell_dofs[c * n_loc + u];
                const double cv = curl[((int64_t)u * 3 + r) * npts + q];
                er += E[2 * (int64_t)g] * cv;
                ei += E[2 * (int64_t)g + 1] * cv;
                lr += lam[2 * (int64_t)g] * cv;
                li += lam[2 * (int64_t)g + 1] * cv;
            }
            const double scale = dim == 2 ? 1.0 / det : hh[r] * hh[r] / det;
            acc += w[q] * scale * (lr * er + li * ei);
        }
    }
    const double m = mu ? mu[c] : 1.0;
    grad[c] = 2.0 * acc / (m * m);
}

void launch_cell_gradient(int dim, int64_t ncells, int n_loc, const FeTables &T, const int32_t *cell_dofs,
                          const double *h, const double *mu, const double *E, const double *lam, double *grad,
                          hipStream_t st) {
    k_cell_grad<<<(unsigned)((ncells + 127) / 128), 128, 0, st>>>(dim, ncells, n_loc, T.npts, T.val.p, T.curl.p,
                                                                  T.w.p, cell_dofs, h, mu, E, lam, grad);
    THM_HIP(hipGetLastError());
}

__global__ void k_sum(const double *x, int64_t n, double *out) {
    __shared__ double red[4];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) a += x[i];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) *out = red[0] + red[1] + red[2] + red[3];
}

void launch_sum(const double *x, int64_t n, double *out, hipStream_t st) {
    k_sum<<<1, 256, 0, st>>>(x, n, out);
    THM_HIP(hipGetLastError());
}

}  // namespace thm
