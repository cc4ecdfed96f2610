// Linear-algebra kernels for gfx950: block SpMV on [[K,-C],[C,K]], Krylov vector
// operations (classical Gram-Schmidt with wave64 reductions, Givens in FP64),
// dense batched GEMM and Gauss-Jordan inversion (preconditioner setup), and the
// block-tridiagonal + static-condensation application of diag(K,K)^{-1}.
//
// Batching: every kernel serves several independent systems.  A flattened block
// schedule maps blockIdx.x to (system, block-in-system) so that systems of very
// different size share one launch without empty blocks.  Vectors of all systems
// live in one arena; system s owns scalars [off[s], off[s] + 2 n_s) of a slot,
// stored as interleaved (re, im) pairs.
#include "kernels.h"

namespace thm {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int find_sys(const int32_t *blkoff, int ns, int b) {
    return blkoff[ns + 1 + b];  // block -> system map stored after the offsets
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block reduction of one double over 256 threads (4 waves); result valid in thread 0.
__device__ __forceinline__ double block_sum256(double v, double *lds) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) lds[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = lds[0] + lds[1] + lds[2] + lds[3];
    return r;
}

template <class T> struct V2;
template <> struct V2<double> { using t = double2; };
template <> struct V2<float> { using t = float2; };

// ------------------------------------------------------------------ SpMV
// y = A x  or  y = b - A x, A = [[K, -sC], [sC, K]] acting on interleaved (re, im)
// pairs, s = +1 (A) or -1 (A^T).  K is read once for both halves.  LPR lanes per row.
template <int LPR, int UNR, class T>
__global__ void __launch_bounds__(256) k_spmv(const MatDesc *__restrict__ mats, const int64_t *__restrict__ off,
                                              const int32_t *__restrict__ blkoff, int ns,
                                              const int32_t *__restrict__ mask, const T *__restrict__ xb,
                                              T *__restrict__ yb, const T *__restrict__ bb, float csign) {
    using T2 = typename V2<T>::t;
    const int s = find_sys(blkoff, ns, blockIdx.x);
    if (mask && !mask[s]) return;
    const MatDesc m = mats[s];
    constexpr int RPB = 256 / LPR;
    const int64_t row = (int64_t)(blockIdx.x - blkoff[s]) * RPB + threadIdx.x / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= m.n) return;
    const T2 *x = reinterpret_cast<const T2 *>(xb + off[s]);
    const T *kv = reinterpret_cast<const T *>(m.kval);
    T ar = 0, ai = 0;
    const int32_t r0 = m.rowptr[row], r1 = m.rowptr[row + 1];
    // UNR entries per lane are loaded before the FMAs (memory-level parallelism).
    int32_t q = r0 + lane;
    if (UNR > 1)
        for (; q + (UNR - 1) * LPR < r1; q += UNR * LPR) {
            T k[UNR];
            int32_t c[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                k[u] = kv[q + u * LPR];
                c[u] = m.col[q + u * LPR];
            }
            T2 xv[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) xv[u] = x[c[u]];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                ar += k[u] * xv[u].x;
                ai += k[u] * xv[u].y;
            }
        }
    for (; q < r1; q += LPR) {
        const T k = kv[q];
        const T2 xv = x[m.col[q]];
        ar += k * xv.x;
        ai += k * xv.y;
    }
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) {
        ar += __shfl_xor(ar, o, LPR);
        ai += __shfl_xor(ai, o, LPR);
    }
    if (lane == 0) {
        const T *cv = reinterpret_cast<const T *>(m.cval);
        const T sg = (T)csign;
        for (int32_t q = m.crowptr[row]; q < m.crowptr[row + 1]; ++q) {
            const T c = sg * cv[q];
            const T2 xv = x[m.ccol[q]];
            ar -= c * xv.y;
            ai += c * xv.x;
        }
        T2 *y = reinterpret_cast<T2 *>(yb + off[s]);
        if (bb) {
            const T2 bv = reinterpret_cast<const T2 *>(bb + off[s])[row];
            y[row] = T2{bv.x - ar, bv.y - ai};
        } else {
            y[row] = T2{ar, ai};
        }
    }
}

// SELL-64 variant: one wave per slice of 64 (length-sorted) rows, one row per lane.  The value and
// column loads of a wave are 64 consecutive entries (coalesced), there is no cross-lane
// reduction and no divergence inside the K loop; padding entries have value 0 and point
// at a valid column.  The boundary operator C (few rows) is applied from its CSR.
template <class T>
__global__ void __launch_bounds__(256) k_spmv_sell(const MatDesc *__restrict__ mats, const int64_t *__restrict__ off,
                                                   const int32_t *__restrict__ blkoff, int ns,
                                                   const int32_t *__restrict__ mask, const T *__restrict__ xb,
                                                   T *__restrict__ yb, const T *__restrict__ bb, float csign) {
    using T2 = typename V2<T>::t;
    const int s = find_sys(blkoff, ns, blockIdx.x);
    if (mask && !mask[s]) return;
    const MatDesc &m = mats[s];
    const int64_t slice = (int64_t)(blockIdx.x - blkoff[s]) * 4 + (threadIdx.x >> 6);
    if (slice * SELL_C >= m.n) return;  // whole wave
    const int lane = threadIdx.x & 63;
    // the matrix (values, columns, row map) and y are touched once per call: non-temporal
    // loads and stores keep them from evicting the gathered entries of x from the caches
    const int32_t row = __builtin_nontemporal_load(m.sl_row + slice * SELL_C + lane);
    const T2 *x = reinterpret_cast<const T2 *>(xb + off[s]);
    const int32_t e0 = m.sl_ptr[slice], w = (m.sl_ptr[slice + 1] - e0) / SELL_C;
    const int32_t *cp = m.sl_col + e0 + lane;
    const T *vp = reinterpret_cast<const T *>(m.sl_val) + e0 + lane;
    T ar = 0, ai = 0;
    int k = 0;
    for (; k + 8 <= w; k += 8) {
        int32_t c[8];
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            c[u] = __builtin_nontemporal_load(cp + (k + u) * SELL_C);
            v[u] = __builtin_nontemporal_load(vp + (k + u) * SELL_C);
        }
        T2 xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) xv[u] = x[c[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            ar += v[u] * xv[u].x;
            ai += v[u] * xv[u].y;
        }
    }
    for (; k < w; ++k) {
        const T v = __builtin_nontemporal_load(vp + k * SELL_C);
        const T2 xv = x[__builtin_nontemporal_load(cp + k * SELL_C)];
        ar += v * xv.x;
        ai += v * xv.y;
    }
    if (row < 0) return;
    const T *cv = reinterpret_cast<const T *>(m.cval);
    const T sg = (T)csign;
    for (int32_t q = m.crowptr[row]; q < m.crowptr[row + 1]; ++q) {
        const T c = sg * cv[q];
        const T2 xv = x[m.ccol[q]];
        ar -= c * xv.y;
        ai += c * xv.x;
    }
    T2 *y = reinterpret_cast<T2 *>(yb + off[s]);
    if (bb) {
        const T2 bv = reinterpret_cast<const T2 *>(bb + off[s])[row];
        ar = bv.x - ar;
        ai = bv.y - ai;
    }
    __builtin_nontemporal_store(ar, &y[row].x);
    __builtin_nontemporal_store(ai, &y[row].y);
}

__global__ void __launch_bounds__(256) k_sell_fill(int64_t ne, const int32_t *__restrict__ src,
                                                   const double *__restrict__ kval, double *__restrict__ v64,
                                                   float *__restrict__ v32) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= ne) return;
    const double v = src[e] >= 0 ? kval[src[e]] : 0.0;
    v64[e] = v;
    v32[e] = (float)v;
}

void launch_sell_fill(int64_t ne, const int32_t *src, const double *kval, double *v64, float *v32, hipStream_t st) {
    if (ne <= 0) return;
    k_sell_fill<<<(unsigned)((ne + 255) / 256), 256, 0, st>>>(ne, src, kval, v64, v32);
    THM_HIP(hipGetLastError());
}

// Variant code v = 10 * lanes_per_row + unroll (unroll 1 or 4), or SPMV_SELL; chosen by
// the autotuner.
template <class T>
void launch_spmv(int v, const MatDesc *mats, const int64_t *off, const Sched &sc, int ns, const int32_t *mask,
                 const T *x, T *y, const T *b, float csign, hipStream_t st) {
    if (!sc.nblocks) return;
    const dim3 g(sc.nblocks), blk(256);
#define SPMV_CASE(L, U) \
    case 10 * L + U: k_spmv<L, U, T><<<g, blk, 0, st>>>(mats, off, sc.blkoff.p, ns, mask, x, y, b, csign); break;
    if (v == SPMV_SELL) {
        k_spmv_sell<T><<<g, blk, 0, st>>>(mats, off, sc.blkoff.p, ns, mask, x, y, b, csign);
        THM_HIP(hipGetLastError());
        return;
    }
    switch (v) {
        SPMV_CASE(2, 1) SPMV_CASE(4, 1) SPMV_CASE(8, 1) SPMV_CASE(16, 1) SPMV_CASE(32, 1) SPMV_CASE(64, 1)
        SPMV_CASE(2, 4) SPMV_CASE(4, 4) SPMV_CASE(8, 4) SPMV_CASE(16, 4) SPMV_CASE(32, 4)
        default: fail(THM_EINVAL, "unknown SpMV variant");
    }
#undef SPMV_CASE
    THM_HIP(hipGetLastError());
}
template void launch_spmv<double>(int, const MatDesc *, const int64_t *, const Sched &, int, const int32_t *,
                                  const double *, double *, const double *, float, hipStream_t);
template void launch_spmv<float>(int, const MatDesc *, const int64_t *, const Sched &, int, const int32_t *,
                                 const float *, float *, const float *, float, hipStream_t);

// Grouped SELL-64 variant: the systems of a group have the same K (pattern and values).
// A slice of 64 rows is served by up to four waves of one block, each applying it to four
// members' vectors (the group's count padded to a multiple of 4; the padding repeats the
// last member and is not stored), so K goes from HBM once per slice and its re-reads by
// the sibling waves hit the caches.  The sum over a row runs in the same order as in
// k_spmv_sell, so both variants give the same bits.  Each member's boundary operator C is
// applied from its own CSR, on the rows where some member has C entries.
// The four members' values of one x entry.  Per-member vectors (IL = false): four gathers.
// Member-interleaved copy (IL = true): the four values are one contiguous 4-complex run.
template <class T, bool IL>
struct GroupX;
template <class T>
struct GroupX<T, false> {
    using T2 = typename V2<T>::t;
    const T2 *x[4];
    __device__ __forceinline__ GroupX(const SpmvGroup &G, int j0, int nmw, const int64_t *off, const T *xb) {
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = reinterpret_cast<const T2 *>(xb + off[G.mem[j0 + min(j, nmw - 1)]]);
    }
    __device__ __forceinline__ void load(int32_t c, T2 (&v)[4]) const {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = x[j][c];
    }
    __device__ __forceinline__ T2 load1(int32_t c, int j) const { return x[j][c]; }
};
template <class T>
struct GroupX<T, true> {
    using T2 = typename V2<T>::t;
    typedef T vec4 __attribute__((ext_vector_type(4)));
    const T *x;
    int64_t ld;  // scalars per row of the interleaved copy
    __device__ __forceinline__ GroupX(const SpmvGroup &G, int j0, int, const int64_t *, const T *xib)
        : x(xib + 2 * (G.xoff + j0)), ld(2 * (int64_t)G.npad) {}
    __device__ __forceinline__ void load(int32_t c, T2 (&v)[4]) const {
        // 8 scalars of members j0 .. j0 + 3 (16-byte aligned: npad, j0 and xoff are multiples of 4)
        const vec4 *p = reinterpret_cast<const vec4 *>(x + c * ld);
        const vec4 a = p[0], b = p[1];
        v[0] = T2{a[0], a[1]};
        v[1] = T2{a[2], a[3]};
        v[2] = T2{b[0], b[1]};
        v[3] = T2{b[2], b[3]};
    }
    __device__ __forceinline__ T2 load1(int32_t c, int j) const {
        return reinterpret_cast<const T2 *>(x + c * ld)[j];
    }
};

template <class T, int U, bool IL>
__device__ __forceinline__ void spmv_group_slice(const MatDesc *__restrict__ mats, const int64_t *__restrict__ off,
                                                 const SpmvGroup &G, int j0, const MatDesc &m, int64_t slice,
                                                 const int32_t *__restrict__ mask, const T *__restrict__ xb,
                                                 T *__restrict__ yb, const T *__restrict__ bb, float csign) {
    using T2 = typename V2<T>::t;
    constexpr int MB = 4;
    const int nmw = min(MB, G.nm - j0);  // members of this wave (1 .. 4)
    const int lane = threadIdx.x & 63;
    const int32_t row = __builtin_nontemporal_load(m.sl_row + slice * SELL_C + lane);
    const int32_t e0 = m.sl_ptr[slice], w = (m.sl_ptr[slice + 1] - e0) / SELL_C;
    const int32_t *cp = m.sl_col + e0 + lane;
    const T *vp = reinterpret_cast<const T *>(m.sl_val) + e0 + lane;
    const GroupX<T, IL> x(G, j0, nmw, off, xb);
    T ar[MB], ai[MB];
#pragma unroll
    for (int j = 0; j < MB; ++j) ar[j] = ai[j] = 0;
    int k = 0;
    for (; k + U <= w; k += U) {
        int32_t c[U];
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = cp[(k + u) * SELL_C];
            v[u] = vp[(k + u) * SELL_C];
        }
        T2 xv[U][MB];
#pragma unroll
        for (int u = 0; u < U; ++u) x.load(c[u], xv[u]);
#pragma unroll
        for (int j = 0; j < MB; ++j)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                ar[j] += v[u] * xv[u][j].x;
                ai[j] += v[u] * xv[u][j].y;
            }
    }
    for (; k < w; ++k) {
        const T v = vp[k * SELL_C];
        const int32_t c = cp[k * SELL_C];
        T2 xv[MB];
        x.load(c, xv);
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            ar[j] += v * xv[j].x;
            ai[j] += v * xv[j].y;
        }
    }
    if (row < 0) return;
    if (G.crow[row]) {
        const T sg = (T)csign;
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            if (j >= nmw) break;
            const MatDesc &mj = mats[G.mem[j0 + j]];
            const T *cv = reinterpret_cast<const T *>(mj.cval);
            for (int32_t q = mj.crowptr[row]; q < mj.crowptr[row + 1]; ++q) {
                const T c = sg * cv[q];
                const T2 xq = x.load1(mj.ccol[q], j);
                ar[j] -= c * xq.y;
                ai[j] += c * xq.x;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < MB; ++j) {
        if (j >= nmw) break;
        const int s = G.mem[j0 + j];
        if (mask && !mask[s]) continue;
        T a = ar[j], b = ai[j];
        if (bb) {
            const T2 bv = reinterpret_cast<const T2 *>(bb + off[s])[row];
            a = bv.x - a;
            b = bv.y - b;
        }
        T2 *y = reinterpret_cast<T2 *>(yb + off[s]);
        __builtin_nontemporal_store(a, &y[row].x);
        __builtin_nontemporal_store(b, &y[row].y);
    }
}

// Block schedule: npad / 4 consecutive waves per slice (see SpmvGroup).  IL: x is the
// member-interleaved copy (see SpmvGroup::xoff) instead of the per-system vectors.
template <class T, bool IL>
__global__ void __launch_bounds__(256) k_spmv_sell_group(const MatDesc *__restrict__ mats,
                                                         const int64_t *__restrict__ off,
                                                         const SpmvGroup *__restrict__ groups,
                                                         const int32_t *__restrict__ blkoff, int ng,
                                                         const int32_t *__restrict__ mask,
                                                         const T *__restrict__ xb, T *__restrict__ yb,
                                                         const T *__restrict__ bb, float csign) {
    const int g = find_sys(blkoff, ng, blockIdx.x);
    const SpmvGroup &G = groups[g];
    const int nmc = G.npad / 4;
    const int64_t gw = (int64_t)(blockIdx.x - blkoff[g]) * 4 + (threadIdx.x >> 6);
    const int64_t slice = gw / nmc;
    const int j0 = 4 * (int)(gw - slice * nmc);
    const MatDesc &m = mats[G.rep];
    if (slice * SELL_C >= m.n) return;  // whole wave
    if (mask) {
        int any = 0;
        for (int j = j0; j < min(j0 + 4, G.nm); ++j) any |= mask[G.mem[j]];
        if (!any) return;
    }
    constexpr int U = sizeof(T) == 4 ? 4 : 2;
    spmv_group_slice<T, U, IL>(mats, off, G, j0, m, slice, mask, xb, yb, bb, csign);
}

template <class T>
void launch_spmv_group(const MatDesc *mats, const int64_t *off, const SpmvGroup *groups, const Sched &sc, int ng,
                       const int32_t *mask, const T *x, T *y, const T *b, float csign, hipStream_t st) {
    if (!sc.nblocks) return;
    k_spmv_sell_group<T, false><<<sc.nblocks, 256, 0, st>>>(mats, off, groups, sc.blkoff.p, ng, mask, x, y, b, csign);
    THM_HIP(hipGetLastError());
}
template <class T>
void launch_spmv_group_i(const MatDesc *mats, const int64_t *off, const SpmvGroup *groups, const Sched &sc, int ng,
                         const int32_t *mask, const T *xi, T *y, float csign, hipStream_t st) {
    if (!sc.nblocks) return;
    k_spmv_sell_group<T, true><<<sc.nblocks, 256, 0, st>>>(mats, off, groups, sc.blkoff.p, ng, mask, xi, y, nullptr,
                                                           csign);
    THM_HIP(hipGetLastError());
}
template void launch_spmv_group_i<double>(const MatDesc *, const int64_t *, const SpmvGroup *, const Sched &, int,
                                          const int32_t *, const double *, double *, float, hipStream_t);
template void launch_spmv_group_i<float>(const MatDesc *, const int64_t *, const SpmvGroup *, const Sched &, int,
                                         const int32_t *, const float *, float *, float, hipStream_t);
template void launch_spmv_group<double>(const MatDesc *, const int64_t *, const SpmvGroup *, const Sched &, int,
                                        const int32_t *, const double *, double *, const double *, float,
                                        hipStream_t);
template void launch_spmv_group<float>(const MatDesc *, const int64_t *, const SpmvGroup *, const Sched &, int,
                                       const int32_t *, const float *, float *, const float *, float, hipStream_t);

// ------------------------------------------------------------------ Krylov vector kernels
// Vectors are interleaved (re, im) pairs.  With cplx = 1 the Arnoldi process uses
// complex scalars (h = <v, w> = sum conj(v) w; the Krylov space is invariant under
// multiplication by i, i.e. the complex GMRES of K + iC expressed on the real block
// vectors); with cplx = 0 it is the real GMRES of the 2N real block system (the
// imaginary part of every inner product is dropped).  Hessenberg, Givens and the
// least-squares solve are FP64 (complex storage in both modes).
// Each block owns VCHUNK scalars of one system and writes one partial per wave.
constexpr int PPT = VCHUNK / 512;  // complex pairs per thread
constexpr int CG = 4;              // basis columns loaded together

// Loads stay unconditional (so the compiler keeps them all in flight): lanes past the
// end of a vector read its last element and their contribution is dropped.
__device__ __forceinline__ int64_t clampi(int64_t i, int64_t np) { return i < np ? i : np - 1; }

template <class T>
__device__ __forceinline__ void wave_store(double v, double *dst) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) *dst = v;
}

template <class T>
__global__ void __launch_bounds__(256) k_dots(const int64_t *__restrict__ off, const int64_t *__restrict__ len,
                                              const int32_t *__restrict__ blkoff, int ns,
                                              const int32_t *__restrict__ mask, const int32_t *__restrict__ jcnt,
                                              const T *__restrict__ V, int64_t ld, const T *__restrict__ w,
                                              double *__restrict__ part, int maxcols, int cplx) {
    using T2 = typename V2<T>::t;
    const int s = find_sys(blkoff, ns, blockIdx.x);
    if (!mask[s]) return;
    const int j = jcnt[s];
    const int64_t base = off[s], np = len[s] / 2;
    const int64_t p0 = (int64_t)(blockIdx.x - blkoff[s]) * (VCHUNK / 2);
    const int wave = threadIdx.x >> 6;
    double *pp = part + ((int64_t)blockIdx.x * NPW + wave) * maxcols;
    T2 wv[PPT];
    const T2 *wp = reinterpret_cast<const T2 *>(w + base);
#pragma unroll
    for (int t = 0; t < PPT; ++t) {
        const int64_t i = p0 + t * 256 + threadIdx.x;
        const T2 x = wp[clampi(i, np)];
        wv[t] = i < np ? x : T2{0, 0};  // zero weight past the end
    }
    // columns in groups of CG: all loads of a group are in flight together
    for (int c0 = 0; c0 <= j; c0 += CG) {
        T2 v[CG][PPT];
#pragma unroll
        for (int u = 0; u < CG; ++u) {
            const T2 *vc = reinterpret_cast<const T2 *>(V + (int64_t)min(c0 + u, j) * ld + base);
#pragma unroll
            for (int t = 0; t < PPT; ++t) v[u][t] = vc[clampi(p0 + t * 256 + threadIdx.x, np)];
        }
#pragma unroll
        for (int u = 0; u < CG; ++u) {
            if (c0 + u > j) break;
            double ar = 0.0, ai = 0.0;
#pragma unroll
            for (int t = 0; t < PPT; ++t) {
                ar += (double)v[u][t].x * (double)wv[t].x + (double)v[u][t].y * (double)wv[t].y;
                ai += (double)v[u][t].x * (double)wv[t].y - (double)v[u][t].y * (double)wv[t].x;
            }
            wave_store<T>(ar, pp + 2 * (c0 + u));
            wave_store<T>(cplx ? ai : 0.0, pp + 2 * (c0 + u) + 1);
        }
    }
}

// out[s][k] (k < ncols) = sum of the partial slots of system s.  Grid (systems,
// column chunks of 16); each wave reduces 4 columns, lanes striding over the slots.
__global__ void k_reduce_cols(const int32_t *__restrict__ blkoff, int ns, const int32_t *__restrict__ mask,
                              const int32_t *__restrict__ jcnt, int ncols_fixed, const double *__restrict__ part,
                              int maxcols, double *__restrict__ out, int ldo, int accumulate) {
    const int s = blockIdx.x;
    if (s >= ns || (mask && !mask[s])) return;
    const int nc = ncols_fixed > 0 ? ncols_fixed : 2 * (jcnt[s] + 1);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b0 = blkoff[s] * NPW, b1 = blkoff[s + 1] * NPW;
    for (int k = 0; k < 4; ++k) {
        const int c = blockIdx.y * 16 + wave * 4 + k;
        if (c >= nc) break;
        double acc = 0.0;
        for (int b = b0 + lane; b < b1; b += 64) acc += part[(int64_t)b * maxcols + c];
        acc = wave_sum(acc);
        if (lane == 0) {
            if (accumulate) out[(int64_t)s * ldo + c] += acc;
            else out[(int64_t)s * ldo + c] = acc;
        }
    }
}

// w -= sum_c V_c h_c (complex h), plus per-wave partial ||w||^2 in column 0.
template <class T>
__global__ void __launch_bounds__(256) k_cgs_update(const int64_t *__restrict__ off, const int64_t *__restrict__ len,
                                                    const int32_t *__restrict__ blkoff, int ns,
                                                    const int32_t *__restrict__ mask, const int32_t *__restrict__ jcnt,
                                                    const T *__restrict__ V, int64_t ld, T *__restrict__ w,
                                                    const double *__restrict__ h, int ldh, double *__restrict__ part,
                                                    int maxcols) {
    using T2 = typename V2<T>::t;
    const int s = find_sys(blkoff, ns, blockIdx.x);
    if (!mask[s]) return;
    const int j = jcnt[s];
    const int64_t base = off[s], np = len[s] / 2;
    const int64_t p0 = (int64_t)(blockIdx.x - blkoff[s]) * (VCHUNK / 2);
    T2 *wp = reinterpret_cast<T2 *>(w + base);
    double xr[PPT], xi[PPT];
#pragma unroll
    for (int t = 0; t < PPT; ++t) {
        const int64_t i = p0 + t * 256 + threadIdx.x;
        const T2 v = wp[clampi(i, np)];
        xr[t] = v.x;
        xi[t] = v.y;
    }
    const double *hs = h + (int64_t)s * ldh;
    for (int c0 = 0; c0 <= j; c0 += CG) {
        T2 v[CG][PPT];
#pragma unroll
        for (int u = 0; u < CG; ++u) {
            const T2 *vc = reinterpret_cast<const T2 *>(V + (int64_t)min(c0 + u, j) * ld + base);
#pragma unroll
            for (int t = 0; t < PPT; ++t) {
                // last read of the basis in this Arnoldi step (the next step streams the
                // preconditioner and the operator first): non-temporal
                typedef T vec2 __attribute__((ext_vector_type(2)));
                const vec2 q = __builtin_nontemporal_load(
                    reinterpret_cast<const vec2 *>(vc + clampi(p0 + t * 256 + threadIdx.x, np)));
                v[u][t] = T2{q.x, q.y};
            }
        }
#pragma unroll
        for (int u = 0; u < CG; ++u) {
            if (c0 + u > j) break;
            const double hr = hs[2 * (c0 + u)], hi = hs[2 * (c0 + u) + 1];
#pragma unroll
            for (int t = 0; t < PPT; ++t) {
                xr[t] -= hr * (double)v[u][t].x - hi * (double)v[u][t].y;
                xi[t] -= hr * (double)v[u][t].y + hi * (double)v[u][t].x;
            }
        }
    }
    double nrm = 0.0;
#pragma unroll
    for (int t = 0; t < PPT; ++t) {
        const int64_t i = p0 + t * 256 + threadIdx.x;
        if (i < np) {
            const T2 v{(T)xr[t], (T)xi[t]};
            wp[i] = v;
            nrm += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        }
    }
    wave_store<T>(nrm, part + ((int64_t)blockIdx.x * NPW + (threadIdx.x >> 6)) * maxcols);
}

// Per-wave partials of ||x||^2.
template <class T>
__global__ void __launch_bounds__(256) k_norm2(const int64_t *__restrict__ off, const int64_t *__restrict__ len,
                                               const int32_t *__restrict__ blkoff, int ns,
                                               const int32_t *__restrict__ mask, const T *__restrict__ x,
                                               double *__restrict__ part, int maxcols) {
    const int s = find_sys(blkoff, ns, blockIdx.x);
    if (mask && !mask[s]) return;
    const int64_t base = off[s], n = len[s];
    const int64_t i0 = (int64_t)(blockIdx.x - blkoff[s]) * VCHUNK;
    double a = 0.0;
#pragma unroll
    for (int t = 0; t < VCHUNK / 256; ++t) {
        const int64_t i = i0 + t * 256 + threadIdx.x;
        const double v = (double)x[base + clampi(i, n)];
        a += i < n ? v * v : 0.0;
    }
    wave_store<T>(a, part + ((int64_t)blockIdx.x * NPW + (threadIdx.x >> 6)) * maxcols);
}

// y = a_s * x (a_s = scal[s] or 1/scal[s]); optional second destination.  The last
// kernel of an Arnoldi step also advances the step counter (step_ctr, one thread).
template <class TI, class TO>
__global__ void __launch_bounds__(256) k_scale(const int64_t *__restrict__ off, const int64_t *__restrict__ len,
                                               const int32_t *__restrict__ blkoff, int ns,
                                               const int32_t *__restrict__ mask, const double *__restrict__ scal,
                                               int invert, const TI *__restrict__ x, TO *__restrict__ y1,
                                               const int32_t *__restrict__ jcol, int64_t ld1, TO *__restrict__ y2,
                                               int32_t *__restrict__ step_ctr) {
    if (step_ctr && blockIdx.x == 0 && threadIdx.x == 0) *step_ctr += 1;
    const int s = find_sys(blkoff, ns, blockIdx.x);
    if (mask && !mask[s]) return;
    const int64_t base = off[s], n = len[s];
    const int64_t i0 = (int64_t)(blockIdx.x - blkoff[s]) * VCHUNK;
    double a = scal ? scal[s] : 1.0;
    if (invert) a = a != 0.0 ? 1.0 / a : 0.0;
    TO *d1 = y1 + base + (jcol ? (int64_t)jcol[s] * ld1 : 0);
#pragma unroll
    for (int t = 0; t < VCHUNK / 256; ++t) {
        const int64_t i = i0 + t * 256 + threadIdx.x;
        const TO v = (TO)(a * (double)x[base + clampi(i, n)]);
        if (i < n) {
            d1[i] = v;
            if (y2) y2[base + i] = v;
        }
    }
}

// y = sum_{c<k} V_c coef[s][c] (complex coefficients), k = kcnt[s].
template <class T>
__global__ void __launch_bounds__(256) k_lincomb(const int64_t *__restrict__ off, const int64_t *__restrict__ len,
                                                 const int32_t *__restrict__ blkoff, int ns,
                                                 const int32_t *__restrict__ mask, const int32_t *__restrict__ kcnt,
                                                 const T *__restrict__ V, int64_t ld, const double *__restrict__ coef,
                                                 int ldc, T *__restrict__ y) {
    using T2 = typename V2<T>::t;
    const int s = find_sys(blkoff, ns, blockIdx.x);
    if (mask && !mask[s]) return;
    const int k = kcnt[s];
    const int64_t base = off[s], np = len[s] / 2;
    const int64_t p0 = (int64_t)(blockIdx.x - blkoff[s]) * (VCHUNK / 2);
    double xr[PPT], xi[PPT];
#pragma unroll
    for (int t = 0; t < PPT; ++t) xr[t] = xi[t] = 0.0;
    for (int c0 = 0; c0 < k; c0 += CG) {
        T2 v[CG][PPT];
#pragma unroll
        for (int u = 0; u < CG; ++u) {
            const T2 *vc = reinterpret_cast<const T2 *>(V + (int64_t)min(c0 + u, k - 1) * ld + base);
#pragma unroll
            for (int t = 0; t < PPT; ++t) v[u][t] = vc[clampi(p0 + t * 256 + threadIdx.x, np)];
        }
#pragma unroll
        for (int u = 0; u < CG; ++u) {
            if (c0 + u >= k) break;
            const double ar = coef[(int64_t)s * ldc + 2 * (c0 + u)], ai = coef[(int64_t)s * ldc + 2 * (c0 + u) + 1];
#pragma unroll
            for (int t = 0; t < PPT; ++t) {
                xr[t] += ar * (double)v[u][t].x - ai * (double)v[u][t].y;
                xi[t] += ar * (double)v[u][t].y + ai * (double)v[u][t].x;
            }
        }
    }
    T2 *yp = reinterpret_cast<T2 *>(y + base);
#pragma unroll
    for (int t = 0; t < PPT; ++t) {
        const int64_t i = p0 + t * 256 + threadIdx.x;
        if (i < np) yp[i] = T2{(T)xr[t], (T)xi[t]};
    }
}

// x += a_s * z (a_s = scal ? scal[s] : 1), x in TX, z in TZ.
template <class TX, class TZ>
__global__ void __launch_bounds__(256) k_axpy(const int64_t *__restrict__ off, const int64_t *__restrict__ len,
                                              const int32_t *__restrict__ blkoff, int ns,
                                              const int32_t *__restrict__ mask, const double *__restrict__ scal,
                                              const TZ *__restrict__ z, TX *__restrict__ x) {
    const int s = find_sys(blkoff, ns, blockIdx.x);
    if (mask && !mask[s]) return;
    const int64_t base = off[s], n = len[s];
    const int64_t i0 = (int64_t)(blockIdx.x - blkoff[s]) * VCHUNK;
    const double a = scal ? scal[s] : 1.0;
#pragma unroll
    for (int t = 0; t < VCHUNK / 256; ++t) {
        const int64_t i = i0 + t * 256 + threadIdx.x;
        const int64_t ic = base + clampi(i, n);
        const TX v = (TX)((double)x[ic] + a * (double)z[ic]);
        if (i < n) x[base + i] = v;
    }
}

__device__ __forceinline__ double slot_sum(const double *part, int maxcols, int b0, int b1, int col) {
    double a = 0.0;
    for (int b = b0 * NPW + (int)threadIdx.x; b < b1 * NPW; b += blockDim.x) a += part[(int64_t)b * maxcols + col];
    return wave_sum(a);  // blockDim.x == 64
}

// Start of a GMRES cycle (one wave per system): beta = ||r||; systems with
// beta/bnorm <= rtol stop; otherwise g = (beta, 0, ...), jcnt = 0, active = 1.  The
// tolerance is read from device memory (the launch may be replayed from a graph); the
// step counter of the cycle is reset; each system's running flag is also written to
// host-visible memory (hrun, may be null).
__global__ void k_cycle_start(int ns, const int32_t *__restrict__ blkoff, const double *__restrict__ part,
                              int maxcols, int32_t *__restrict__ running, int32_t *__restrict__ active,
                              int32_t *__restrict__ jcnt, const double *__restrict__ bnorm,
                              const double *__restrict__ rtol_d, double *__restrict__ g, int m,
                              double *__restrict__ beta_out, double *__restrict__ resid_out,
                              int32_t *__restrict__ iters, int max_iter, int32_t *__restrict__ step_ctr,
                              int32_t *__restrict__ hrun) {
    const int s = blockIdx.x;
    if (s >= ns) return;
    if (s == 0 && threadIdx.x == 0 && step_ctr) *step_ctr = 0;
    if (!running[s]) {
        if (threadIdx.x == 0) {
            active[s] = 0;
            if (hrun) hrun[s] = 0;
        }
        return;
    }
    const double rtol = *rtol_d;
    const double beta = sqrt(slot_sum(part, maxcols, blkoff[s], blkoff[s + 1], 0));
    double *gs = g + (int64_t)s * 2 * (m + 1);
    for (int i = threadIdx.x; i < 2 * (m + 1); i += blockDim.x) gs[i] = 0.0;
    if (threadIdx.x != 0) return;
    const double rel = bnorm[s] > 0.0 ? beta / bnorm[s] : 0.0;
    resid_out[s] = rel;
    beta_out[s] = beta;
    jcnt[s] = 0;
    if (!(rel > rtol) || iters[s] >= max_iter || !isfinite(rel)) {
        running[s] = 0;
        active[s] = 0;
        if (hrun) hrun[s] = 0;
        return;
    }
    active[s] = 1;
    if (hrun) hrun[s] = 1;
    gs[0] = beta;
}

// After Arnoldi step j (one wave per system): h_{j+1,j} = ||w||, apply the previous
// complex Givens rotations to column j of H, build the new one, update g.
// Rotation G = [[c, s], [-conj(s), c]] with c real: G [a; b] = [r; 0].
__global__ void k_arnoldi_finish(int ns, const int32_t *__restrict__ blkoff, const double *__restrict__ part,
                                 int maxcols, int32_t *__restrict__ active, int32_t *__restrict__ jcnt,
                                 const double *__restrict__ hcol, int ldh, double *__restrict__ H,
                                 double *__restrict__ cs, double *__restrict__ sn, double *__restrict__ g,
                                 double *__restrict__ hnext, const double *__restrict__ bnorm,
                                 const double *__restrict__ rtol_d, int m, int32_t *__restrict__ iters, int max_iter,
                                 double *__restrict__ resid_est, int32_t *__restrict__ hflags,
                                 const int32_t *__restrict__ step_ctr, int spc, int nslots) {
    __shared__ double colr[1025], coli[1025], csl[1024], snr[1024], sni[1024];
    const int s = blockIdx.x;
    if (s >= ns) return;
    // the system's flag after this step, also written to host memory (one slot per group of
    // spc consecutive steps: the last step of the group leaves its flag there)
    int32_t *hf = hflags + (int64_t)((*step_ctr / spc) % nslots) * ns + s;
    if (!active[s]) {
        if (threadIdx.x == 0) *hf = 0;
        return;
    }
    const int j = jcnt[s];
    const double hn = sqrt(slot_sum(part, maxcols, blkoff[s], blkoff[s + 1], 0));
    const double *hc = hcol + (int64_t)s * ldh;
    double *css = cs + (int64_t)s * m, *sns = sn + (int64_t)s * 2 * m;
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        colr[i] = hc[2 * i];
        coli[i] = hc[2 * i + 1];
        if (i < j) {
            csl[i] = css[i];
            snr[i] = sns[2 * i];
            sni[i] = sns[2 * i + 1];
        }
    }
    __syncthreads();
    double *gs = g + (int64_t)s * 2 * (m + 1);
    if (threadIdx.x == 0) {
        const double br = hn, bi = 0.0;  // entry j+1 of the column (real on input)
        colr[j + 1] = br;
        coli[j + 1] = bi;
        // The rotated entry i+1 of one rotation is entry i of the next: it stays in registers,
        // so the chain of rotations carries no LDS store-to-load round trip.
        double xr = colr[0], xi = coli[0];
        for (int i = 0; i < j; ++i) {
            const double c = csl[i], sr = snr[i], si = sni[i];
            const double ar = xr, ai = xi, cr = colr[i + 1], ci = coli[i + 1];
            // t = c a + s b ;  b' = -conj(s) a + c b
            colr[i] = c * ar + (sr * cr - si * ci);
            coli[i] = c * ai + (sr * ci + si * cr);
            xr = -(sr * ar + si * ai) + c * cr;
            xi = -(sr * ai - si * ar) + c * ci;
        }
        colr[j] = xr;
        coli[j] = xi;
        const double ar = xr, ai = xi, bnr = colr[j + 1], bni = coli[j + 1];
        const double na = hypot(ar, ai), nb = hypot(bnr, bni);
        const double den = hypot(na, nb);
        double c = 1.0, sr = 0.0, si = 0.0, rr = ar, ri = ai;
        if (den > 0.0) {
            if (na == 0.0) {
                c = 0.0; sr = 1.0; si = 0.0; rr = bnr; ri = bni;  // rotation maps b to the top
                // with a = 0: [c a + s b] = b, and -conj(s) a + c b = 0
            } else {
                const double ur = ar / na, ui = ai / na;  // a/|a|
                c = na / den;
                // s = (a/|a|) conj(b) / den
                sr = (ur * bnr + ui * bni) / den;
                si = (ui * bnr - ur * bni) / den;
                rr = ur * den;
                ri = ui * den;
            }
        }
        css[j] = c;
        sns[2 * j] = sr;
        sns[2 * j + 1] = si;
        colr[j] = rr;
        coli[j] = ri;
        colr[j + 1] = 0.0;
        coli[j + 1] = 0.0;
        // g_{j+1} = -conj(s) g_j ; g_j = c g_j
        const double gr = gs[2 * j], gi = gs[2 * j + 1];
        gs[2 * (j + 1)] = -(sr * gr + si * gi);
        gs[2 * (j + 1) + 1] = -(sr * gi - si * gr);
        gs[2 * j] = c * gr;
        gs[2 * j + 1] = c * gi;
        hnext[s] = hn;
        jcnt[s] = j + 1;
        iters[s] += 1;
        const double est = hypot(gs[2 * (j + 1)], gs[2 * (j + 1) + 1]) / bnorm[s];
        resid_est[s] = est;
        const bool breakdown = !(hn > 1e-300) || !(den > 0.0);
        const int32_t on = !(est <= *rtol_d || breakdown || j + 1 >= m || iters[s] >= max_iter || !isfinite(est));
        active[s] = on;
        *hf = on;
    }
    __syncthreads();
    double *Hs = H + (int64_t)s * 2 * (m + 1) * m + (int64_t)j * 2 * (m + 1);  // column j, complex
    for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) {
        Hs[2 * i] = colr[i];
        Hs[2 * i + 1] = coli[i];
    }
}

// y = H^{-1} g on the first k = jcnt[s] columns (upper triangular, complex); one wave
// per system, column-oriented back substitution.
__global__ void k_hsolve(int ns, const int32_t *__restrict__ running, const int32_t *__restrict__ jcnt,
                         const double *__restrict__ H, const double *__restrict__ g, double *__restrict__ y, int m) {
    __shared__ double rr[1025], ri[1025];
    const int s = blockIdx.x;
    if (s >= ns || !running[s]) return;
    const int k = jcnt[s];
    const double *Hs = H + (int64_t)s * 2 * (m + 1) * m;
    const double *gs = g + (int64_t)s * 2 * (m + 1);
    double *ys = y + (int64_t)s * 2 * (m + 1);
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        rr[i] = gs[2 * i];
        ri[i] = gs[2 * i + 1];
    }
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
        const double *col = Hs + (int64_t)i * 2 * (m + 1);
        const double dr = col[2 * i], di = col[2 * i + 1];
        const double den = dr * dr + di * di;
        // y_i = r_i / d
        const double yr = den > 0.0 ? (rr[i] * dr + ri[i] * di) / den : 0.0;
        const double yi = den > 0.0 ? (ri[i] * dr - rr[i] * di) / den : 0.0;
        for (int r = threadIdx.x; r < i; r += blockDim.x) {
            const double hr = col[2 * r], hi = col[2 * r + 1];
            rr[r] -= hr * yr - hi * yi;
            ri[r] -= hr * yi + hi * yr;
        }
        if (threadIdx.x == 0) {
            ys[2 * i] = yr;
            ys[2 * i + 1] = yi;
        }
        __syncthreads();
    }
}

// Zero the entries flagged in `dir` (Dirichlet rows) of a complex vector.
template <class T>
__global__ void k_zero_flagged(const int64_t *__restrict__ off, const int64_t *__restrict__ nvec,
                               const int32_t *__restrict__ blkoff, int ns, const uint8_t *const *__restrict__ dirs,
                               T *__restrict__ x) {
    const int s = find_sys(blkoff, ns, blockIdx.x);
    const int64_t i = (int64_t)(blockIdx.x - blkoff[s]) * 256 + threadIdx.x;
    if (i >= nvec[s]) return;
    if (dirs[s][i]) { x[off[s] + 2 * i] = (T)0; x[off[s] + 2 * i + 1] = (T)0; }
}

// out[s] = sqrt(sum of partials); with bnorm: resid[s] = out/bnorm, running[s] = 0 if <= rtol.
__global__ void k_norm_finish(int ns, const int32_t *__restrict__ blkoff, const double *__restrict__ part,
                              int maxcols, const int32_t *__restrict__ mask, double *__restrict__ out,
                              const double *__restrict__ bnorm, double rtol, double *__restrict__ resid,
                              int32_t *__restrict__ running) {
    const int s = blockIdx.x;
    if (s >= ns || (mask && !mask[s])) return;
    const double nrm = sqrt(slot_sum(part, maxcols, blkoff[s], blkoff[s + 1], 0));
    if (threadIdx.x != 0) return;
    out[s] = nrm;
    if (bnorm) {
        const double rel = bnorm[s] > 0.0 ? nrm / bnorm[s] : 0.0;
        resid[s] = rel;
        if (running && !(rel > rtol)) running[s] = 0;
    }
}

// ------------------------------------------------------------------ launchers
#define VGRID(sc) dim3((sc).nblocks), dim3(256), 0, st
#define VGUARD(B) if (!(B).vs.nblocks) return

template <class T>
void launch_dots(const Batch &B, const int32_t *mask, const int32_t *jcnt, const T *V, int64_t ld, const T *w,
                 double *part, int cplx, hipStream_t st) {
    VGUARD(B);
    k_dots<T><<<VGRID(B.vs)>>>(B.off.p, B.len.p, B.vs.blkoff.p, B.ns, mask, jcnt, V, ld, w, part, B.maxcols, cplx);
    THM_HIP(hipGetLastError());
}
template <class T>
void launch_cgs_update(const Batch &B, const int32_t *mask, const int32_t *jcnt, const T *V, int64_t ld, T *w,
                       const double *h, int ldh, double *part, hipStream_t st) {
    VGUARD(B);
    k_cgs_update<T><<<VGRID(B.vs)>>>(B.off.p, B.len.p, B.vs.blkoff.p, B.ns, mask, jcnt, V, ld, w, h, ldh, part,
                                     B.maxcols);
    THM_HIP(hipGetLastError());
}
template <class T>
void launch_norm2(const Batch &B, const int32_t *mask, const T *x, double *part, hipStream_t st) {
    VGUARD(B);
    k_norm2<T><<<VGRID(B.vs)>>>(B.off.p, B.len.p, B.vs.blkoff.p, B.ns, mask, x, part, B.maxcols);
    THM_HIP(hipGetLastError());
}
template <class TI, class TO>
void launch_scale(const Batch &B, const int32_t *mask, const double *scal, int invert, const TI *x, TO *y1,
                  const int32_t *jcol, int64_t ld1, TO *y2, hipStream_t st, int32_t *step_ctr) {
    VGUARD(B);
    k_scale<TI, TO><<<VGRID(B.vs)>>>(B.off.p, B.len.p, B.vs.blkoff.p, B.ns, mask, scal, invert, x, y1, jcol, ld1, y2,
                                     step_ctr);
    THM_HIP(hipGetLastError());
}
template <class T>
void launch_lincomb(const Batch &B, const int32_t *mask, const int32_t *kcnt, const T *V, int64_t ld,
                    const double *coef, int ldc, T *y, hipStream_t st) {
    VGUARD(B);
    k_lincomb<T><<<VGRID(B.vs)>>>(B.off.p, B.len.p, B.vs.blkoff.p, B.ns, mask, kcnt, V, ld, coef, ldc, y);
    THM_HIP(hipGetLastError());
}
template <class TX, class TZ>
void launch_axpy(const Batch &B, const int32_t *mask, const double *scal, const TZ *z, TX *x, hipStream_t st) {
    VGUARD(B);
    k_axpy<TX, TZ><<<VGRID(B.vs)>>>(B.off.p, B.len.p, B.vs.blkoff.p, B.ns, mask, scal, z, x);
    THM_HIP(hipGetLastError());
}
void launch_norm_finish(const Batch &B, const double *part, const int32_t *mask, double *out, const double *bnorm,
                        double rtol, double *resid, int32_t *running, hipStream_t st) {
    k_norm_finish<<<B.ns, 64, 0, st>>>(B.ns, B.vs.blkoff.p, part, B.maxcols, mask, out, bnorm, rtol,
                                                   resid, running);
    THM_HIP(hipGetLastError());
}
void launch_reduce_cols(const Batch &B, const int32_t *mask, const int32_t *jcnt, int ncols_fixed,
                        const double *part, double *out, int ldo, int accumulate, hipStream_t st) {
    const int chunks = ncols_fixed > 0 ? (ncols_fixed + 15) / 16 : (B.maxcols + 15) / 16;
    k_reduce_cols<<<dim3(B.ns, chunks), 256, 0, st>>>(B.vs.blkoff.p, B.ns, mask, jcnt, ncols_fixed, part, B.maxcols, out, ldo,
                                       accumulate);
    THM_HIP(hipGetLastError());
}
void launch_cycle_start(const Batch &B, const double *part, int32_t *running, int32_t *active, int32_t *jcnt,
                        const double *bnorm, const double *rtol_d, double *g, int m, double *beta, double *resid,
                        int32_t *iters, int max_iter, int32_t *step_ctr, int32_t *hrun, hipStream_t st) {
    k_cycle_start<<<B.ns, 64, 0, st>>>(B.ns, B.vs.blkoff.p, part, B.maxcols, running, active, jcnt, bnorm, rtol_d,
                                       g, m, beta, resid, iters, max_iter, step_ctr, hrun);
    THM_HIP(hipGetLastError());
}
void launch_arnoldi_finish(const Batch &B, const double *part, int32_t *active, int32_t *jcnt, const double *hcol,
                           int ldh, double *H, double *cs, double *sn, double *g, double *hnext,
                           const double *bnorm, const double *rtol_d, int m, int32_t *iters, int max_iter,
                           double *est, int32_t *hflags, const int32_t *step_ctr, int spc, int nslots,
                           hipStream_t st) {
    if (m > 1024) fail(THM_EINVAL, "restart must be <= 1024");
    k_arnoldi_finish<<<B.ns, 64, 0, st>>>(B.ns, B.vs.blkoff.p, part, B.maxcols, active, jcnt, hcol,
                                                      ldh, H, cs, sn, g, hnext, bnorm, rtol_d, m, iters, max_iter,
                                                      est, hflags, step_ctr, spc, nslots);
    THM_HIP(hipGetLastError());
}
void launch_hsolve(const Batch &B, const int32_t *running, const int32_t *jcnt, const double *H, const double *g,
                   double *y, int m, hipStream_t st) {
    k_hsolve<<<B.ns, 64, 0, st>>>(B.ns, running, jcnt, H, g, y, m);
    THM_HIP(hipGetLastError());
}
template <class T>
void launch_zero_flagged(const Batch &B, const uint8_t *const *dirs, T *x, hipStream_t st) {
    if (!B.es.nblocks) return;
    k_zero_flagged<T><<<B.es.nblocks, 256, 0, st>>>(B.off.p, B.nvec.p, B.es.blkoff.p, B.ns, dirs, x);
    THM_HIP(hipGetLastError());
}

#define INST_T(T)                                                                                            \
    template void launch_dots<T>(const Batch &, const int32_t *, const int32_t *, const T *, int64_t,         \
                                 const T *, double *, int, hipStream_t);                                     \
    template void launch_cgs_update<T>(const Batch &, const int32_t *, const int32_t *, const T *, int64_t,   \
                                       T *, const double *, int, double *, hipStream_t);                     \
    template void launch_norm2<T>(const Batch &, const int32_t *, const T *, double *, hipStream_t);          \
    template void launch_lincomb<T>(const Batch &, const int32_t *, const int32_t *, const T *, int64_t,      \
                                    const double *, int, T *, hipStream_t);                                  \
    template void launch_zero_flagged<T>(const Batch &, const uint8_t *const *, T *, hipStream_t);
INST_T(double)
INST_T(float)
template void launch_scale<double, double>(const Batch &, const int32_t *, const double *, int, const double *,
                                           double *, const int32_t *, int64_t, double *, hipStream_t, int32_t *);
template void launch_scale<float, float>(const Batch &, const int32_t *, const double *, int, const float *,
                                         float *, const int32_t *, int64_t, float *, hipStream_t, int32_t *);
template void launch_scale<float, double>(const Batch &, const int32_t *, const double *, int, const float *,
                                          double *, const int32_t *, int64_t, double *, hipStream_t, int32_t *);
template void launch_scale<double, float>(const Batch &, const int32_t *, const double *, int, const double *,
                                          float *, const int32_t *, int64_t, float *, hipStream_t, int32_t *);
template void launch_axpy<double, double>(const Batch &, const int32_t *, const double *, const double *, double *,
                                          hipStream_t);
template void launch_axpy<float, float>(const Batch &, const int32_t *, const double *, const float *, float *,
                                        hipStream_t);
template void launch_axpy<double, float>(const Batch &, const int32_t *, const double *, const float *, double *,
                                         hipStream_t);

}  // namespace thm
