// The complete inverse (K + iC)^{-1} of a subdomain system, applied through the exact
// factorised K^{-1} and a low-rank correction (Sec. 3.2 names the complete inverse of
// the block system as the alternative to the block-diagonal preconditioner of eq. (11)).
//
// C is nonzero only on the r boundary DoFs Gamma (impedance and transmission sides), so
// C = P^T C_G P with P the restriction to Gamma and C_G its r x r block.  With
// S_G = P K^{-1} P^T and M = I + i C_G S_G (Woodbury):
//     (K + iC)^{-1} b = z - K^{-1} P^T M^{-1} (i C_G P z),     z = K^{-1} b.
// For the transposed system (K - iC) the signs of i flip and M^{-1} is conjugated.
// Setup (FP64): columns of S_G from batched applications of K^{-1} to unit vectors, the
// real 2r x 2r form [[I, -C_G S_G], [C_G S_G, I]] of M, its inverse by Gauss-Jordan, and
// M^{-1} stored complex, column-major, FP64 and FP32.
//
// Vectors follow the batch layout of the Krylov kernels: system s owns scalars
// [off[s], off[s] + 2 n_s), interleaved (re, im).  Per-system Gamma quantities are
// concatenated: entries [goff[s], goff[s + 1]) belong to system s (r_s of them).
#include "kernels.h"

namespace thm {

// ------------------------------------------------------------------ setup
// x[gamma_s[2k]].re = val, x[gamma_s[2k + 1]].im = val for every selected system, with
// k = k0 + kadd[s] (kadd may be null: k = k0).
__global__ void k_full_unit(int ns, const int32_t *__restrict__ mask, const int64_t *__restrict__ goff,
                            const int32_t *__restrict__ gam, const int64_t *__restrict__ off,
                            const int32_t *__restrict__ kadd, int k0, double val, double *__restrict__ x) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns || (mask && !mask[s])) return;
    const int64_t g0 = goff[s], r = goff[s + 1] - g0;
    const int64_t k = k0 + (kadd ? kadd[s] : 0);
    if (2 * k < r) x[off[s] + 2 * (int64_t)gam[g0 + 2 * k]] = val;
    if (2 * k + 1 < r) x[off[s] + 2 * (int64_t)gam[g0 + 2 * k + 1] + 1] = val;
}

// Columns 2k and 2k + 1 of S_G (column-major r x r at soff[s]) from z = K^{-1} x, with
// k = k0 + kadd[s] as above.
__global__ void k_full_gather(int ns, const int32_t *__restrict__ mask, const int64_t *__restrict__ goff,
                              const int32_t *__restrict__ gam, const int64_t *__restrict__ off,
                              const int32_t *__restrict__ kadd, int k0, const double *__restrict__ z,
                              const int64_t *__restrict__ soff, double *__restrict__ S) {
    const int s = blockIdx.y;
    if (mask && !mask[s]) return;
    const int64_t g0 = goff[s], r = goff[s + 1] - g0;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= r) return;
    const int64_t k = k0 + (kadd ? kadd[s] : 0);
    const double *zs = z + off[s] + 2 * (int64_t)gam[g0 + i];
    double *Ss = S + soff[s];
    if (2 * k < r) Ss[(2 * k) * r + i] = zs[0];
    if (2 * k + 1 < r) Ss[(2 * k + 1) * r + i] = zs[1];
}

// Real form of M = I + i C_G S_G for one system: Bm = [[I, -Q], [Q, I]], Q = C_G S_G,
// row-major 2r x 2r.  C_G rows: cptr[i] .. cptr[i + 1] over (ccol, cval), Gamma-local.
__global__ void k_full_block(int r, const double *__restrict__ S, const int32_t *__restrict__ cptr,
                             const int32_t *__restrict__ ccol, const double *__restrict__ cval,
                             double *__restrict__ Bm) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)r * r) return;
    const int i = (int)(e / r), j = (int)(e % r);
    double q = 0.0;
    for (int32_t t = cptr[i]; t < cptr[i + 1]; ++t) q += cval[t] * S[(int64_t)j * r + ccol[t]];
    const int64_t n2 = 2 * (int64_t)r;
    const double d = i == j ? 1.0 : 0.0;
    Bm[i * n2 + j] = d;
    Bm[i * n2 + r + j] = -q;
    Bm[(r + i) * n2 + j] = q;
    Bm[(r + i) * n2 + r + j] = d;
}

// M^{-1} from the inverse of the real form (its first block column holds Re and Im),
// stored complex column-major in FP64 and FP32.
__global__ void k_full_extract(int r, const double *__restrict__ Inv, double *__restrict__ M64,
                               float *__restrict__ M32) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)r * r) return;
    const int i = (int)(e / r), j = (int)(e % r);
    const int64_t n2 = 2 * (int64_t)r;
    const double re = Inv[i * n2 + j], im = Inv[(r + i) * n2 + j];
    const int64_t o = 2 * ((int64_t)j * r + i);
    M64[o] = re;
    M64[o + 1] = im;
    M32[o] = (float)re;
    M32[o + 1] = (float)im;
}

// ------------------------------------------------------------------ apply
// u = (+-i) C_G z_G per system (complex; conj selects -i).
template <class T>
__global__ void __launch_bounds__(256) k_full_u(int ns, const int32_t *__restrict__ mask,
                                                const int64_t *__restrict__ goff, const int32_t *__restrict__ gam,
                                                const int32_t *__restrict__ cptr, const int32_t *__restrict__ ccol,
                                                const T *__restrict__ cval, const int64_t *__restrict__ off,
                                                const T *__restrict__ z, int conj, T *__restrict__ u) {
    const int s = blockIdx.y;
    if (mask && !mask[s]) return;
    const int64_t g0 = goff[s], r = goff[s + 1] - g0;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= r) return;
    const T *zs = z + off[s];
    double ar = 0.0, ai = 0.0;
    for (int32_t t = cptr[g0 + i]; t < cptr[g0 + i + 1]; ++t) {
        const double c = (double)cval[t];
        const int64_t p = 2 * (int64_t)gam[g0 + ccol[t]];
        ar += c * (double)zs[p];
        ai += c * (double)zs[p + 1];
    }
    // i (ar + i ai) = -ai + i ar ;  -i (ar + i ai) = ai - i ar
    u[2 * (g0 + i)] = (T)(conj ? ai : -ai);
    u[2 * (g0 + i) + 1] = (T)(conj ? -ar : ar);
}

constexpr int FULL_CW = 64;  // columns of M^{-1} per block (one LDS chunk of u)

// Partial products of t = M^{-1} u: block (row tile of 256, column chunk c) of system s
// writes part[(g0 + i) * nchmax + c].  M^{-1} column-major, so consecutive threads read
// consecutive complex entries of one column.
template <class T>
__global__ void __launch_bounds__(256) k_full_mv(int ns, const int32_t *__restrict__ mask,
                                                 const int64_t *__restrict__ goff, const int64_t *__restrict__ moff,
                                                 const T *__restrict__ M, const T *__restrict__ u, int nchmax,
                                                 int conj, T *__restrict__ part) {
    __shared__ T ul[2 * FULL_CW];
    const int s = blockIdx.y;
    if (mask && !mask[s]) return;
    const int64_t g0 = goff[s];
    const int r = (int)(goff[s + 1] - g0);
    if (r == 0) return;  // no boundary DoFs: nothing to correct (same for the whole block)
    const int ntile = (r + 255) / 256;
    const int tile = blockIdx.x % ntile, c = blockIdx.x / ntile;
    const int j0 = c * FULL_CW;
    if (blockIdx.x >= ntile * ((r + FULL_CW - 1) / FULL_CW)) return;  // same for the whole block
    const int jn = min(FULL_CW, r - j0);
    if (threadIdx.x < 2 * jn) ul[threadIdx.x] = u[2 * (g0 + j0) + threadIdx.x];
    __syncthreads();
    const int i = tile * 256 + threadIdx.x;
    if (i >= r) return;
    const T *Ms = M + 2 * moff[s];
    const double sg = conj ? -1.0 : 1.0;
    double ar = 0.0, ai = 0.0;
    for (int j = 0; j < jn; ++j) {
        const int64_t o = 2 * ((int64_t)(j0 + j) * r + i);
        const double mr = (double)Ms[o], mi = sg * (double)Ms[o + 1];
        const double ur = (double)ul[2 * j], ui = (double)ul[2 * j + 1];
        ar += mr * ur - mi * ui;
        ai += mr * ui + mi * ur;
    }
    part[2 * ((g0 + i) * nchmax + c)] = (T)ar;
    part[2 * ((g0 + i) * nchmax + c) + 1] = (T)ai;
}

// t = sum of the partials; w[gamma_i] = t (w is zero outside Gamma).
template <class T>
__global__ void __launch_bounds__(256) k_full_fin(int ns, const int32_t *__restrict__ mask,
                                                  const int64_t *__restrict__ goff, const int32_t *__restrict__ gam,
                                                  const int64_t *__restrict__ off, const T *__restrict__ part,
                                                  int nchmax, T *__restrict__ w) {
    const int s = blockIdx.y;
    if (mask && !mask[s]) return;
    const int64_t g0 = goff[s], r = goff[s + 1] - g0;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= r) return;
    const int nch = (int)((r + FULL_CW - 1) / FULL_CW);
    double ar = 0.0, ai = 0.0;
    for (int c = 0; c < nch; ++c) {
        ar += (double)part[2 * ((g0 + i) * nchmax + c)];
        ai += (double)part[2 * ((g0 + i) * nchmax + c) + 1];
    }
    T *ws = w + off[s] + 2 * (int64_t)gam[g0 + i];
    ws[0] = (T)ar;
    ws[1] = (T)ai;
}

// ------------------------------------------------------------------ launchers
void launch_full_unit(const FullDesc &F, int ns, const int32_t *mask, const int64_t *off, const int32_t *kadd,
                      int k, double val, double *x, hipStream_t st) {
    k_full_unit<<<(ns + 63) / 64, 64, 0, st>>>(ns, mask, F.goff, F.gam, off, kadd, k, val, x);
    THM_HIP(hipGetLastError());
}

void launch_full_gather(const FullDesc &F, int ns, const int32_t *mask, const int64_t *off, const int32_t *kadd,
                        int k, const double *z, const int64_t *soff, double *S, hipStream_t st) {
    if (!F.maxr || !ns) return;
    k_full_gather<<<dim3((F.maxr + 255) / 256, ns), 256, 0, st>>>(ns, mask, F.goff, F.gam, off, kadd, k, z, soff,
                                                                  S);
    THM_HIP(hipGetLastError());
}

void launch_full_block(int r, const double *S, const int32_t *cptr, const int32_t *ccol, const double *cval,
                       double *Bm, hipStream_t st) {
    const int64_t n = (int64_t)r * r;
    if (!n) return;
    k_full_block<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(r, S, cptr, ccol, cval, Bm);
    THM_HIP(hipGetLastError());
}

void launch_full_extract(int r, const double *Inv, double *M64, float *M32, hipStream_t st) {
    const int64_t n = (int64_t)r * r;
    if (!n) return;
    k_full_extract<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(r, Inv, M64, M32);
    THM_HIP(hipGetLastError());
}

template <class T>
void launch_full_correct(const FullDesc &F, int ns, const int32_t *mask, const int64_t *off, int conj, const T *z,
                         T *u, T *part, T *w, hipStream_t st) {
    if (!F.maxr || !ns) return;
    const T *cval = static_cast<const T *>(sizeof(T) == 8 ? F.cval64 : F.cval32);
    const T *M = static_cast<const T *>(sizeof(T) == 8 ? F.m64 : F.m32);
    const int rt = (F.maxr + 255) / 256;
    k_full_u<T><<<dim3(rt, ns), 256, 0, st>>>(ns, mask, F.goff, F.gam, F.cptr, F.ccol, cval, off, z, conj, u);
    k_full_mv<T><<<dim3(rt * F.nchmax, ns), 256, 0, st>>>(ns, mask, F.goff, F.moff, M, u, F.nchmax, conj, part);
    k_full_fin<T><<<dim3(rt, ns), 256, 0, st>>>(ns, mask, F.goff, F.gam, off, part, F.nchmax, w);
    THM_HIP(hipGetLastError());
}
template void launch_full_correct<double>(const FullDesc &, int, const int32_t *, const int64_t *, int,
                                          const double *, double *, double *, double *, hipStream_t);
template void launch_full_correct<float>(const FullDesc &, int, const int32_t *, const int64_t *, int,
                                         const float *, float *, float *, float *, hipStream_t);

}  // namespace thm
