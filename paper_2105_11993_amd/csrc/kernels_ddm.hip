// Domain-decomposition kernels (eqs. (6)-(10), transmission operator S = 1) and
// small vector kernels used by the boundary projection.
//
// Interface data are FP64 complex dual vectors G_{i->j} on the non-Dirichlet DoFs
// of the closure of Sigma_ij.  Subdomain i's right-hand side receives -G_{j->i};
// the update is G_{i->j} = -G_{j->i} - 2 i k w M_Sigma_ij E_i.
#include "kernels.h"

namespace thm {

// rhs_s[dof] = base_s[dof] (or 0) - sum of incoming interface data at that DoF.
__global__ void k_ddm_rhs(int64_t ntouch, const int32_t *__restrict__ touch_sys, const int32_t *__restrict__ touch_dof,
                          const int32_t *__restrict__ touch_ptr, const int32_t *__restrict__ touch_src,
                          double *const *__restrict__ rhs, const double *__restrict__ G) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntouch) return;
    double re = 0.0, im = 0.0;
    for (int32_t e = touch_ptr[t]; e < touch_ptr[t + 1]; ++e) {
        re += G[2 * (int64_t)touch_src[e]];
        im += G[2 * (int64_t)touch_src[e] + 1];
    }
    double *r = rhs[touch_sys[t]] + 2 * (int64_t)touch_dof[t];
    r[0] -= re;
    r[1] -= im;
}

void launch_ddm_rhs(int64_t ntouch, const int32_t *touch_sys, const int32_t *touch_dof, const int32_t *touch_ptr,
                    const int32_t *touch_src, double *const *rhs, const double *G, hipStream_t st) {
    if (!ntouch) return;
    k_ddm_rhs<<<(unsigned)((ntouch + 255) / 256), 256, 0, st>>>(ntouch, touch_sys, touch_dof, touch_ptr, touch_src,
                                                                rhs, G);
    THM_HIP(hipGetLastError());
}

// For every directed-interface entry e (sender s, local row la), transmission S = s 1:
//   u_e = -G[rev(e)] - 2 i k w s (M_Sigma E_s)[la]
//   mode 0: out_e = u_e          (Jacobi sweep / affine term b)
//   mode 1: out_e = G_e - u_e    ((I - A0) G)
__global__ void k_ddm_update(int64_t nent, const int32_t *__restrict__ ent_sys, const int32_t *__restrict__ ent_row,
                             const int32_t *__restrict__ ent_rev, const int32_t *__restrict__ ent_mptr,
                             const int32_t *__restrict__ m_col, const double *__restrict__ m_val,
                             const double *const *__restrict__ X, const double *__restrict__ G, double kw,
                             double s_re, double s_im, int mode, double *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nent) return;
    const double *Es = X[ent_sys[e]];
    double mr = 0.0, mi = 0.0;
    for (int32_t q = ent_mptr[e]; q < ent_mptr[e + 1]; ++q) {
        const double v = m_val[q];
        const int64_t c = m_col[q];
        mr += v * Es[2 * c];
        mi += v * Es[2 * c + 1];
    }
    (void)ent_row;
    const int64_t r = ent_rev[e];
    // t = s (mr + i mi);  -2 i kw t = 2 kw Im(t) - 2 i kw Re(t)
    const double tr = s_re * mr - s_im * mi, ti = s_re * mi + s_im * mr;
    const double ur = -G[2 * r] + 2.0 * kw * ti;
    const double ui = -G[2 * r + 1] - 2.0 * kw * tr;
    if (mode == 0) {
        out[2 * e] = ur;
        out[2 * e + 1] = ui;
    } else {
        out[2 * e] = G[2 * e] - ur;
        out[2 * e + 1] = G[2 * e + 1] - ui;
    }
}

void launch_ddm_update(int64_t nent, const int32_t *ent_sys, const int32_t *ent_row, const int32_t *ent_rev,
                       const int32_t *ent_mptr, const int32_t *m_col, const double *m_val,
                       const double *const *X, const double *G, double kw, double s_re, double s_im, int mode,
                       double *out, hipStream_t st) {
    if (!nent) return;
    k_ddm_update<<<(unsigned)((nent + 255) / 256), 256, 0, st>>>(nent, ent_sys, ent_row, ent_rev, ent_mptr, m_col,
                                                                 m_val, X, G, kw, s_re, s_im, mode, out);
    THM_HIP(hipGetLastError());
}

// Glue: E[g] = X_owner(g)[loc(g)] (owner = lowest subdomain id holding g).
__global__ void k_ddm_glue(int64_t n, const int32_t *__restrict__ own_sys, const int32_t *__restrict__ own_loc,
                           const double *const *__restrict__ X, double *__restrict__ E) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const double *src = X[own_sys[g]] + 2 * (int64_t)own_loc[g];
    E[2 * g] = src[0];
    E[2 * g + 1] = src[1];
}

void launch_ddm_glue(int64_t n, const int32_t *own_sys, const int32_t *own_loc, const double *const *X, double *E,
                     hipStream_t st) {
    k_ddm_glue<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, own_sys, own_loc, X, E);
    THM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- Jacobi-PCG helpers (single system)
// z = r ./ d  (complex r, real diagonal d; entries with d == 0 -> 0)
__global__ void k_diag_solve(int64_t n, const double *d, const double *r, double *z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double inv = d[i] != 0.0 ? 1.0 / d[i] : 0.0;
    z[2 * i] = r[2 * i] * inv;
    z[2 * i + 1] = r[2 * i + 1] * inv;
}
void launch_diag_solve(int64_t n, const double *d, const double *r, double *z, hipStream_t st) {
    k_diag_solve<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, d, r, z);
    THM_HIP(hipGetLastError());
}

// dot = sum a_i b_i over 2n scalars (single block grid-stride, deterministic)
__global__ void k_dot1(int64_t m, const double *a, const double *b, double *out) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) acc += a[i] * b[i];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) *out = red[0] + red[1] + red[2] + red[3];
}
void launch_dot1(int64_t m, const double *a, const double *b, double *out, hipStream_t st) {
    k_dot1<<<1, 256, 0, st>>>(m, a, b, out);
    THM_HIP(hipGetLastError());
}

// y = a*x + b*y with a = sa[0] (or -sa[0] if neg), b = sb ? sb[0] : 1 ... scalar ratios from device:
// mode 0: x += (num/den) p ; r -= (num/den) q     (CG update, sc = {num, den})
// mode 1: p = z + (num/den) p                     (sc = {num_new, num_old})
__global__ void k_cg_step(int64_t m, int mode, const double *sc, double *x, const double *p, double *r,
                          const double *q, double *pp, const double *z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const double a = sc[1] != 0.0 ? sc[0] / sc[1] : 0.0;
    if (mode == 0) {
        x[i] += a * p[i];
        r[i] -= a * q[i];
    } else {
        pp[i] = z[i] + a * pp[i];
    }
}
void launch_cg_step(int64_t m, int mode, const double *sc, double *x, const double *p, double *r, const double *q,
                    double *pp, const double *z, hipStream_t st) {
    k_cg_step<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(m, mode, sc, x, p, r, q, pp, z);
    THM_HIP(hipGetLastError());
}

}  // namespace thm
