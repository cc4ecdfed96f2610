// Batched blocked Gauss-Jordan inversion with partial pivoting (setup of the cyclic-
// reduction factor and of the complete-inverse correction).
//
// The matrix is inverted in place in panels of GJ_NB columns.  Inside a panel every
// column is eliminated as in the unblocked method (pivot search over the rows not yet
// pivoted, the row swap applied to whole rows, the elimination applied to every row but
// only to the panel's columns).  The other columns receive the panel's elimination at
// once, as two products with the panel's rows r and columns c:
//     A[not r, not c] += A[not r, c] A[r, not c]        (old A[r, not c])
//     A[r, not c]      = A[r, c] A[r, not c]
// The row swaps make the result the inverse of the row-permuted matrix; its columns are
// permuted back at the end.  Work per matrix is one rank-GJ_NB product per panel instead
// of one pass over the whole matrix per column.
#include "kernels.h"

namespace thm {

constexpr int GJ_NB = 64;

__device__ __forceinline__ int find_sys2(const int32_t *blkoff, int nd, int b) {
    return blkoff[nd + 1 + b];  // block -> matrix map stored after the offsets
}

// pivot row of column col: largest magnitude among rows col..n-1 (lowest index on ties)
__global__ void k_bgj_pivot(const InvDesc *ds, int nd, int col, int32_t *status) {
    __shared__ double bv[256];
    __shared__ int bi[256];
    const int di = blockIdx.x;
    if (di >= nd) return;
    const InvDesc d = ds[di];
    if (col >= d.n) return;
    double best = -1.0;
    int bidx = col;
    for (int i = col + threadIdx.x; i < d.n; i += blockDim.x) {
        const double v = fabs(d.A[(int64_t)i * d.n + col]);
        if (v > best) {
            best = v;
            bidx = i;
        }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = bidx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double v2 = bv[threadIdx.x + o];
            const int i2 = bi[threadIdx.x + o];
            if (v2 > bv[threadIdx.x] || (v2 == bv[threadIdx.x] && i2 < bi[threadIdx.x])) {
                bv[threadIdx.x] = v2;
                bi[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        d.piv[col] = bi[0];
        if (!(bv[0] > 0.0) || !isfinite(bv[0])) atomicOr(status, 1);
    }
}

// swap rows col and piv[col] (whole rows), then copy the pivot row's panel entries and
// the pivot column into per-matrix scratch (prow: GJ_NB values, pcol: n values)
__global__ void __launch_bounds__(256) k_bgj_swap(const InvDesc *ds, int nd, int col) {
    const int di = blockIdx.y;
    const InvDesc d = ds[di];
    if (col >= d.n) return;
    const int p = d.piv[col];
    if (p == col) return;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= d.n) return;
    double *a = d.A + (int64_t)col * d.n + j, *b = d.A + (int64_t)p * d.n + j;
    const double t = *a;
    *a = *b;
    *b = t;
}

__global__ void __launch_bounds__(256) k_bgj_gather(const InvDesc *ds, int nd, const int64_t *soff, int col, int kb,
                                                    double *scr) {
    const int di = blockIdx.y;
    const InvDesc d = ds[di];
    if (col >= d.n) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double *prow = scr + soff[di], *pcol = prow + GJ_NB;
    if (i < d.n) pcol[i] = d.A[i * d.n + col];
    if (i < GJ_NB && kb + i < d.n) prow[i] = d.A[(int64_t)col * d.n + kb + i];
}

// elimination of column col on the panel's columns [kb, kb + w) of every row
__global__ void __launch_bounds__(256) k_bgj_panel(const InvDesc *__restrict__ ds, const int32_t *__restrict__ blkoff,
                                                   int nd, const int64_t *__restrict__ soff, int col, int kb,
                                                   const double *__restrict__ scr) {
    const int di = find_sys2(blkoff, nd, blockIdx.x);
    const InvDesc d = ds[di];
    const int n = d.n;
    if (col >= n) return;
    const int64_t e = (int64_t)(blockIdx.x - blkoff[di]) * 256 + threadIdx.x;
    const int i = (int)(e / GJ_NB), jj = (int)(e % GJ_NB);
    const int j = kb + jj;
    if (i >= n || j >= n || j >= kb + GJ_NB) return;
    const double *prow = scr + soff[di], *pcol = prow + GJ_NB;
    const double pv = pcol[col];
    const double ipv = pv != 0.0 ? 1.0 / pv : 0.0;
    const double pr = (j == col) ? ipv : prow[jj] * ipv;
    double out;
    if (i == col) {
        out = pr;
    } else {
        const double f = pcol[i];
        const double ev = (j == col) ? 0.0 : d.A[(int64_t)i * n + j];
        out = ev - f * pr;
    }
    d.A[(int64_t)i * n + j] = out;
}

// A[r, not c] = T (the product A[r, c] A[r, not c], staged in W) for the panel rows r
__global__ void __launch_bounds__(256) k_bgj_copyback(const InvDesc *__restrict__ ds, const int32_t *__restrict__ blkoff,
                                                      int nd, int kb) {
    const int di = find_sys2(blkoff, nd, blockIdx.x);
    const InvDesc d = ds[di];
    const int n = d.n;
    const int w = min(GJ_NB, n - kb);
    const int64_t e = (int64_t)(blockIdx.x - blkoff[di]) * 256 + threadIdx.x;
    if (w <= 0 || e >= (int64_t)w * n) return;
    const int r = (int)(e / n), j = (int)(e % n);
    if (j >= kb && j < kb + w) return;
    d.A[(int64_t)(kb + r) * n + j] = d.W[(int64_t)r * n + j];
}

__global__ void k_bgj_perm_build(const InvDesc *ds, int nd) {
    const int di = blockIdx.x * blockDim.x + threadIdx.x;
    if (di >= nd) return;
    const InvDesc d = ds[di];
    int32_t *perm = d.piv + d.n;
    for (int j = 0; j < d.n; ++j) perm[j] = j;
    for (int c = d.n - 1; c >= 0; --c) {
        const int p = d.piv[c];
        const int32_t t = perm[c];
        perm[c] = perm[p];
        perm[p] = t;
    }
}

__global__ void __launch_bounds__(256) k_bgj_perm_apply(const InvDesc *__restrict__ ds,
                                                        const int32_t *__restrict__ blkoff, int nd) {
    const int di = find_sys2(blkoff, nd, blockIdx.x);
    const InvDesc d = ds[di];
    const int n = d.n;
    const int nch = (n + 255) / 256;
    const int local = blockIdx.x - blkoff[di];
    const int i = local / nch;
    const int j = (local - i * nch) * 256 + threadIdx.x;
    if (i >= n || j >= n) return;
    d.out[(int64_t)i * d.ldo + j] = d.A[(int64_t)i * n + d.piv[n + j]];
}

void launch_invert_blocked(const std::vector<InvDesc> &d, int32_t *status, hipStream_t st) {
    if (d.empty()) return;
    const int nd = (int)d.size();
    int nmax = 0;
    std::vector<int64_t> soff(nd), units_panel(nd), units_perm(nd), units_copy(nd);
    int64_t stot = 0;
    for (int i = 0; i < nd; ++i) {
        nmax = std::max(nmax, d[i].n);
        soff[i] = stot;
        stot += GJ_NB + d[i].n;
        units_panel[i] = (int64_t)d[i].n * GJ_NB;
        units_perm[i] = (int64_t)d[i].n * ((d[i].n + 255) / 256);
        units_copy[i] = (int64_t)d[i].n * GJ_NB;
    }
    DBuf<InvDesc> dd;
    dd.upload(d, st);
    DBuf<int64_t> dsoff;
    dsoff.upload(soff, st);
    DBuf<double> scr(stot);
    Sched sp, sperm, scopy;
    sp.build(units_panel, 256, st);
    scopy.build(units_copy, 256, st);
    sperm.build(units_perm, 1, st);
    DBuf<GemmDesc> gscr;
    Sched gsched;
    const unsigned rb = (unsigned)((nmax + 255) / 256);
    for (int kb = 0; kb < nmax; kb += GJ_NB) {
        const int kend = std::min(nmax, kb + GJ_NB);
        for (int col = kb; col < kend; ++col) {
            k_bgj_pivot<<<nd, 256, 0, st>>>(dd.p, nd, col, status);
            k_bgj_swap<<<dim3(rb, nd), 256, 0, st>>>(dd.p, nd, col);
            k_bgj_gather<<<dim3(rb, nd), 256, 0, st>>>(dd.p, nd, dsoff.p, col, kb, scr.p);
            k_bgj_panel<<<sp.nblocks, 256, 0, st>>>(dd.p, sp.blkoff.p, nd, dsoff.p, col, kb, scr.p);
        }
        THM_HIP(hipGetLastError());
        // rank-w updates of the columns outside the panel
        std::vector<GemmDesc> g;
        for (int i = 0; i < nd; ++i) {
            const int n = d[i].n;
            if (kb >= n) continue;
            const int w = std::min(GJ_NB, n - kb);
            const int lo[2] = {0, kb + w}, len[2] = {kb, n - kb - w};
            double *A = d[i].A;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    if (!len[a] || !len[b]) continue;
                    // A[I, J] += A[I, panel] A[panel, J]
                    g.push_back({len[a], len[b], w, 0, 0, A + (int64_t)lo[a] * n + kb, A + (int64_t)kb * n + lo[b],
                                 A + (int64_t)lo[a] * n + lo[b], n, n, n, 1.0, 1.0});
                }
            for (int b = 0; b < 2; ++b) {
                if (!len[b]) continue;
                // W[0:w, J] = A[panel, panel] A[panel, J]
                g.push_back({w, len[b], w, 0, 0, A + (int64_t)kb * n + kb, A + (int64_t)kb * n + lo[b],
                             d[i].W + lo[b], n, n, n, 1.0, 0.0});
            }
        }
        launch_gemm_batched(g, st, gscr, gsched);
        k_bgj_copyback<<<scopy.nblocks, 256, 0, st>>>(dd.p, scopy.blkoff.p, nd, kb);
        THM_HIP(hipGetLastError());
    }
    k_bgj_perm_build<<<(nd + 63) / 64, 64, 0, st>>>(dd.p, nd);
    k_bgj_perm_apply<<<sperm.nblocks, 256, 0, st>>>(dd.p, sperm.blkoff.p, nd);
    THM_HIP(hipGetLastError());
    THM_HIP(hipStreamSynchronize(st));  // keeps the schedules and scratch alive until the kernels finished
}

}  // namespace thm
