// Block preconditioner diag(K, K)^{-1} of eq. (11) with an exact factorised K^{-1}:
//  1. static condensation of the cell-interior DoFs (per-cell dense inverse),
//  2. block cyclic reduction of the block-tridiagonal system on the skeleton
//     (edge/face) DoFs, layered along the last axis: every level eliminates the
//     odd-positioned blocks (explicit dense inverses) and couples the even ones.
// Application to the two right-hand sides (real and imaginary halves) is one
// batched MFMA launch per level and direction; systems whose matrices are identical
// share one factor, and their right-hand sides become extra columns of one product.
#include "kernels.h"

namespace thm {

__device__ __forceinline__ int find_sys2(const int32_t *blkoff, int ns, int b) {
    return blkoff[ns + 1 + b];  // block -> system map stored after the offsets
}

template <class T> struct P2;
template <> struct P2<double> { using t = double2; };
template <> struct P2<float> { using t = float2; };

// ------------------------------------------------------------------ condensation (setup)
// One block per cell: K'_c = K_c with Dirichlet rows/columns zeroed; Kii^{-1} by
// Gauss-Jordan with partial pivoting; F = K'_ei Kii^{-1}; Kcond = K'_ee - F K'_ie.
__global__ void __launch_bounds__(256) k_condense(int n_loc, int n_int, const double *__restrict__ Kel,
                                                  const int32_t *__restrict__ cell_dofs,
                                                  const uint8_t *__restrict__ dir, double *__restrict__ kiinv,
                                                  double *__restrict__ Fout, double *__restrict__ Kcond,
                                                  int32_t *status) {
    __shared__ double Kc[64 * 64];
    __shared__ double Ai[32 * 32];
    __shared__ double prow[32], fcol[32];
    __shared__ int perm[32], pivs[32];
    __shared__ uint8_t dl[64];
    const int64_t c = blockIdx.x;
    const int tid = threadIdx.x;
    const int ne = n_loc - n_int;
    for (int u = tid; u < n_loc; u += blockDim.x) dl[u] = dir[cell_dofs[c * n_loc + u]];
    __syncthreads();
    for (int id = tid; id < n_loc * n_loc; id += blockDim.x) {
        const int u = id / n_loc, v = id % n_loc;
        Kc[id] = (dl[u] || dl[v]) ? 0.0 : Kel[c * n_loc * n_loc + id];
    }
    __syncthreads();
    if (n_int > 0) {
        for (int id = tid; id < n_int * n_int; id += blockDim.x) {
            const int i = id / n_int, j = id % n_int;
            Ai[id] = Kc[(ne + i) * n_loc + ne + j];
        }
        __syncthreads();
        for (int col = 0; col < n_int; ++col) {
            if (tid == 0) {
                int p = col;
                double best = fabs(Ai[col * n_int + col]);
                for (int i = col + 1; i < n_int; ++i) {
                    const double v = fabs(Ai[i * n_int + col]);
                    if (v > best) { best = v; p = i; }
                }
                pivs[col] = p;
                if (!(best > 0.0) || !isfinite(best)) atomicOr(status, 1);
            }
            __syncthreads();
            const int p = pivs[col];
            if (p != col)
                for (int j = tid; j < n_int; j += blockDim.x) {
                    const double t = Ai[col * n_int + j];
                    Ai[col * n_int + j] = Ai[p * n_int + j];
                    Ai[p * n_int + j] = t;
                }
            __syncthreads();
            const double pv = Ai[col * n_int + col];
            const double ipv = pv != 0.0 ? 1.0 / pv : 0.0;
            for (int j = tid; j < n_int; j += blockDim.x) {
                prow[j] = (j == col) ? ipv : Ai[col * n_int + j] * ipv;
                fcol[j] = Ai[j * n_int + col];
            }
            __syncthreads();
            for (int id = tid; id < n_int * n_int; id += blockDim.x) {
                const int i = id / n_int, j = id % n_int;
                if (i == col) Ai[id] = prow[j];
                else Ai[id] = (j == col ? 0.0 : Ai[id]) - fcol[i] * prow[j];
            }
            __syncthreads();
        }
        // undo the row interchanges as column swaps in reverse order
        if (tid == 0) {
            for (int j = 0; j < n_int; ++j) perm[j] = j;
            for (int col = n_int - 1; col >= 0; --col) {
                const int p = pivs[col];
                const int t = perm[col];
                perm[col] = perm[p];
                perm[p] = t;
            }
        }
        __syncthreads();
        for (int id = tid; id < n_int * n_int; id += blockDim.x) {
            const int i = id / n_int, j = id % n_int;
            kiinv[c * n_int * n_int + id] = Ai[i * n_int + perm[j]];
        }
        __syncthreads();
        for (int id = tid; id < n_int * n_int; id += blockDim.x) Ai[id] = kiinv[c * n_int * n_int + id];
        __syncthreads();
        // F = K'_ei Kii^{-1} (ne x n_int)
        for (int id = tid; id < ne * n_int; id += blockDim.x) {
            const int u = id / n_int, m = id % n_int;
            double acc = 0.0;
            for (int k = 0; k < n_int; ++k) acc += Kc[u * n_loc + ne + k] * Ai[k * n_int + m];
            Fout[c * ne * n_int + id] = acc;
        }
        __syncthreads();
    }
    for (int id = tid; id < ne * ne; id += blockDim.x) {
        const int u = id / ne, v = id % ne;
        double acc = Kc[u * n_loc + v];
        for (int m = 0; m < n_int; ++m) acc -= Fout[c * ne * n_int + u * n_int + m] * Kc[(ne + m) * n_loc + v];
        Kcond[c * ne * ne + id] = acc;
    }
}

void launch_condense(int ncells, int n_loc, int n_int, const double *Kel, const int32_t *cell_dofs,
                     const uint8_t *dir, double *kiinv, double *F, double *Kcond, int32_t *status, hipStream_t st) {
    if (n_loc > 64 || n_int > 32) fail(THM_EUNSUPPORTED, "condensation supports n_loc <= 64 and n_int <= 32");
    k_condense<<<ncells, 256, 0, st>>>(n_loc, n_int, Kel, cell_dofs, dir, kiinv, F, Kcond, status);
    THM_HIP(hipGetLastError());
}

__global__ void k_fill(double *p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
void launch_fill(double *p, int64_t n, double v, hipStream_t st) {
    if (!n) return;
    k_fill<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, n, v);
    THM_HIP(hipGetLastError());
}

__global__ void k_tgt_gather(int64_t ntgt, const int64_t *tgt_index, const int32_t *tgt_kind, const int32_t *tgt_ptr,
                             const int32_t *tgt_src, const double *Kcond, double *sinv, double *lf) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntgt) return;
    double acc = 0.0;
    for (int32_t e = tgt_ptr[t]; e < tgt_ptr[t + 1]; ++e) acc += Kcond[tgt_src[e]];
    (tgt_kind[t] ? lf : sinv)[tgt_index[t]] = acc;
}
void launch_tgt_gather(int64_t ntgt, const int64_t *tgt_index, const int32_t *tgt_kind, const int32_t *tgt_ptr,
                       const int32_t *tgt_src, const double *Kcond, double *sinv, double *lf, hipStream_t st) {
    if (!ntgt) return;
    k_tgt_gather<<<(unsigned)((ntgt + 255) / 256), 256, 0, st>>>(ntgt, tgt_index, tgt_kind, tgt_ptr, tgt_src, Kcond,
                                                                 sinv, lf);
    THM_HIP(hipGetLastError());
}

__global__ void k_dir_identity(int64_t n_skel, const int32_t *skel_dof, const uint8_t *dir, const int64_t *boff,
                               const int64_t *sinv_off, const int32_t *bsize, int nlayers, double *sinv) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_skel || !dir[skel_dof[t]]) return;
    int lo = 0, hi = nlayers;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (boff[mid] <= t) lo = mid; else hi = mid;
    }
    const int64_t i = t - boff[lo];
    sinv[sinv_off[lo] + i * bsize[lo] + i] = 1.0;
}
void launch_dir_identity(int64_t n_skel, const int32_t *skel_dof, const uint8_t *dir, const int64_t *boff,
                         const int64_t *sinv_off, const int32_t *bsize, int nlayers, double *sinv, hipStream_t st) {
    k_dir_identity<<<(unsigned)((n_skel + 255) / 256), 256, 0, st>>>(n_skel, skel_dof, dir, boff, sinv_off, bsize,
                                                                     nlayers, sinv);
    THM_HIP(hipGetLastError());
}

__global__ void k_transpose(const double *A, int m, int n, int lda, double *At, int ldt, double alpha) {
    __shared__ double t[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;  // 32 x 8 threads
    for (int r = ty; r < 32; r += 8) {
        const int i = by + r, j = bx + tx;
        if (i < m && j < n) t[r][tx] = A[(int64_t)i * lda + j];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int j = bx + r, i = by + tx;
        if (i < m && j < n) At[(int64_t)j * ldt + i] = alpha * t[tx][r];
    }
}
void launch_transpose(const double *A, int m, int n, int lda, double *At, int ldt, double alpha, hipStream_t st) {
    if (!m || !n) return;
    dim3 g((n + 31) / 32, (m + 31) / 32);
    k_transpose<<<g, 256, 0, st>>>(A, m, n, lda, At, ldt, alpha);
    THM_HIP(hipGetLastError());
}

// mismatch[0] |= (a != b) over n entries (bitwise comparison of double arrays)
__global__ void k_compare(const uint64_t *a, const uint64_t *b, int64_t n, int32_t *mismatch) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && a[i] != b[i]) *mismatch = 1;
}
void launch_compare(const void *a, const void *b, int64_t nbytes8, int32_t *mismatch, hipStream_t st) {
    if (!nbytes8) return;
    k_compare<<<(unsigned)((nbytes8 + 255) / 256), 256, 0, st>>>((const uint64_t *)a, (const uint64_t *)b, nbytes8,
                                                                 mismatch);
    THM_HIP(hipGetLastError());
}

__global__ void k_convert(const double *a, float *b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}
void launch_convert(const double *a, float *b, int64_t n, hipStream_t st) {
    if (!n) return;
    k_convert<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(a, b, n);
    THM_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ application (batched)
// Condensation terms: tw[c ne + le] = (F_c r_int(c))[le], one thread per cell and
// skeleton local DoF (the 12-24 interior values of a cell are read by its ne threads).
template <class T>
__global__ void __launch_bounds__(256) k_cond_fr(const PrecDesc *__restrict__ pd, const int64_t *__restrict__ off,
                                                 const int64_t *__restrict__ toff, const int32_t *__restrict__ blkoff,
                                                 int ns, const int32_t *__restrict__ mask, const T *__restrict__ rb,
                                                 T *__restrict__ twb) {
    using T2 = typename P2<T>::t;
    const int s = find_sys2(blkoff, ns, blockIdx.x);
    if (mask && !mask[s]) return;
    const PrecDesc &d = pd[s];
    const int64_t e = (int64_t)(blockIdx.x - blkoff[s]) * 256 + threadIdx.x;
    if (e >= (int64_t)d.n_cells * d.ne) return;
    const int64_t c = e / d.ne;
    const int le = (int)(e - c * d.ne);
    const T *f = reinterpret_cast<const T *>(d.FT) + c * d.n_int * d.ne + le;  // F^T[c][m][le]
    const T2 *ri = reinterpret_cast<const T2 *>(rb + off[s]) + d.cell_off + c * d.n_int;
    T2 acc{0, 0};
#pragma unroll 4
    for (int m = 0; m < d.n_int; ++m) {
        const T fv = f[(int64_t)m * d.ne];
        const T2 rv = ri[m];
        acc.x += fv * rv.x;
        acc.y += fv * rv.y;
    }
    reinterpret_cast<T2 *>(twb)[toff[s] + e] = acc;
}

// ws[t] = r[skel_dof[t]] - sum over the cells c of t of (F_c r_int(c))[local t], stored at
// the padded position of the system's member columns (see wv_pos).
template <class T>
__global__ void __launch_bounds__(256) k_cond_fwd(const PrecDesc *__restrict__ pd, const int64_t *__restrict__ off,
                                                  const int64_t *__restrict__ soff, const int64_t *__restrict__ toff,
                                                  const int32_t *__restrict__ blkoff, int ns,
                                                  const int32_t *__restrict__ mask, const T *__restrict__ rb,
                                                  const T *__restrict__ twb, T *__restrict__ wsb) {
    using T2 = typename P2<T>::t;
    const int s = find_sys2(blkoff, ns, blockIdx.x);
    if (mask && !mask[s]) return;
    const PrecDesc &d = pd[s];
    const int64_t t = (int64_t)(blockIdx.x - blkoff[s]) * 256 + threadIdx.x;
    if (t >= d.n_skel) return;
    const T2 *r = reinterpret_cast<const T2 *>(rb + off[s]);
    const T2 *tw = reinterpret_cast<const T2 *>(twb) + toff[s];
    T *ws = wsb + soff[s];  // the system's real column; the imaginary one starts 8 later
    T2 acc = r[d.skel_dof[t]];
    if (d.n_int > 0)
        for (int32_t e = d.cond_ptr[t]; e < d.cond_ptr[t + 1]; ++e) {
            const T2 v = tw[(int64_t)d.cond_cell[e] * d.ne + d.cond_loc[e]];
            acc.x -= v.x;
            acc.y -= v.y;
        }
    T *wp = ws + wv_pos(d.skel_pos[t], d.cs);
    wp[0] = acc.x;
    wp[8] = acc.y;
}

// ------------------------------------------------------------------ cyclic-reduction apply (MFMA)
// Every task is a dense product Y = M X: M is rows x ld (one cyclic-reduction block:
// an inverse and/or couplings), X holds the task's input segments of every member of
// the factor group as columns (real and imaginary part of each member are separate
// columns, so 8 members fill one 16-wide n tile).
//   subtract = 1:  y[row] = y[row] - (M X)[row]   (reduction of the right-hand side)
//   subtract = 0:  y[row] =          (M X)[row]   (back substitution / last blocks)
// A block owns 32 rows (two 16 x 16 MFMA tiles) and up to 16 members; its waves split
// the columns into contiguous ranges and the partial tiles are summed through LDS in a
// fixed order, so the result does not depend on scheduling.  Within a 32-column step,
// lane group g (lanes 16 g .. 16 g + 15) feeds the MFMA k index g, row i16 of M and
// column i16 of X; its value j (j = h P + t, P = 16 / sizeof(T) values per 16-byte
// piece) is step column bcr_col(g, j) = 4 P h + P g + t.  The four lane groups thus read
// 64 contiguous bytes of a row of M or of a column of X per load instruction.  The sum
// over k is order-free, so this permutation is exact.
template <class T> struct Mfma;
// Both forms take A[i][k] from lane i + 16 k and B[k][j] from lane j + 16 k; they
// differ in where accumulator v of lane j + 16 g sits: row 4 g + v (f32) or row
// g + 4 v (f64).
template <> struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
};
template <> struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int v) { return g + 4 * v; }
};

// ------------------------------------------------------------------ batched FP64 GEMM (setup)
// C = alpha op(A) op(B) + beta C for a batch of matrices: 64 x 64 tiles of C per block, 32-deep
// K steps staged through LDS, each wave a 32 x 32 quarter of the tile as 2 x 2 MFMA tiles
// (v_mfma_f64_16x16x4f64: lane i + 16 g feeds A[i][k0 + g] and B[k0 + g][i]).  The next K
// step's operands are loaded into registers while the current one runs on the matrix cores;
// each operand is read along its contiguous direction (per transpose flag).  The order of the
// sum over k is fixed (k ascending in steps of 4), so results are reproducible.
constexpr int GEMM_BK = 32;
__global__ void __launch_bounds__(256) k_gemm(const GemmDesc *__restrict__ ds, const int32_t *__restrict__ blkoff,
                                              int nd) {
    using V4 = Mfma<double>::v4;
    __shared__ double As[GEMM_BK][64 + 1];
    __shared__ double Bs[GEMM_BK][64 + 1];
    const int di = find_sys2(blkoff, nd, blockIdx.x);
    const GemmDesc d = ds[di];
    const int tiles_n = (d.n + 63) / 64;
    const int tile = blockIdx.x - blkoff[di];
    const int tm = tile / tiles_n, tn = tile % tiles_n;
    const int row0 = tm * 64, col0 = tn * 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i16 = lane & 15, g = lane >> 4;
    const int wr = 32 * (wave >> 1), wc = 32 * (wave & 1);
    constexpr int NPT = GEMM_BK * 64 / 256;  // operand values per thread and step
    // (row, k) of value q of this thread in the A tile and (k, col) in the B tile: consecutive
    // threads take consecutive addresses of the stored operand
    auto a_at = [&](int q, int &r, int &kk) {
        const int e = (int)threadIdx.x + 256 * q;
        if (d.ta) { r = e % 64; kk = e / 64; } else { r = e / GEMM_BK; kk = e % GEMM_BK; }
    };
    auto b_at = [&](int q, int &kk, int &c) {
        const int e = (int)threadIdx.x + 256 * q;
        if (d.tb) { kk = e % GEMM_BK; c = e / GEMM_BK; } else { kk = e / 64; c = e % 64; }
    };
    double ra[NPT], rb[NPT];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            int r, kk;
            a_at(q, r, kk);
            const int gi = row0 + r, gk = k0 + kk;
            ra[q] = (gi < d.m && gk < d.k) ? (d.ta ? d.A[(int64_t)gk * d.lda + gi] : d.A[(int64_t)gi * d.lda + gk])
                                           : 0.0;
            int kb, c;
            b_at(q, kb, c);
            const int gk2 = k0 + kb, gj = col0 + c;
            rb[q] = (gk2 < d.k && gj < d.n) ? (d.tb ? d.B[(int64_t)gj * d.ldb + gk2] : d.B[(int64_t)gk2 * d.ldb + gj])
                                            : 0.0;
        }
    };
    V4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = V4{0.0, 0.0, 0.0, 0.0};
    fetch(0);
    for (int k0 = 0; k0 < d.k; k0 += GEMM_BK) {
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            int r, kk;
            a_at(q, r, kk);
            As[kk][r] = ra[q];
            int kb, c;
            b_at(q, kb, c);
            Bs[kb][c] = rb[q];
        }
        __syncthreads();
        if (k0 + GEMM_BK < d.k) fetch(k0 + GEMM_BK);  // in flight while this step runs
#pragma unroll
        for (int k4 = 0; k4 < GEMM_BK; k4 += 4) {
            double a2[2], b2[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                a2[t] = As[k4 + g][wr + 16 * t + i16];
                b2[t] = Bs[k4 + g][wc + 16 * t + i16];
            }
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = Mfma<double>::op(a2[mt], b2[nt], acc[mt][nt]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = row0 + wr + 16 * mt + Mfma<double>::row(g, v);
                const int gj = col0 + wc + 16 * nt + i16;
                if (gi >= d.m || gj >= d.n) continue;
                double *cp = d.C + (int64_t)gi * d.ldc + gj;
                *cp = d.alpha * acc[mt][nt][v] + (d.beta != 0.0 ? d.beta * *cp : 0.0);
            }
}

void launch_gemm_batched(const std::vector<GemmDesc> &g, hipStream_t st, DBuf<GemmDesc> &scratch, Sched &sched) {
    if (g.empty()) return;
    std::vector<int64_t> tiles(g.size());
    for (size_t i = 0; i < g.size(); ++i) tiles[i] = (int64_t)((g[i].m + 63) / 64) * ((g[i].n + 63) / 64);
    sched.build(tiles, 1, st);
    scratch.upload(g, st);
    if (sched.nblocks == 0) return;
    k_gemm<<<sched.nblocks, 256, 0, st>>>(scratch.p, sched.blkoff.p, (int)g.size());
    THM_HIP(hipGetLastError());
}

// Values per 16-byte piece, and the step column that value j of lane group g carries.
static_assert(BCR_RT == 32 && BCR_KS == 32, "the lane order of a tile assumes 32 x 32 tiles");
template <class T> constexpr int bcr_per() { return 16 / (int)sizeof(T); }
template <class T>
__host__ __device__ constexpr int bcr_col(int g, int j) {
    return 4 * bcr_per<T>() * (j / bcr_per<T>()) + bcr_per<T>() * g + j % bcr_per<T>();
}

// One 16-byte aligned piece from global memory: v[h P .. h P + P) = p[0 .. P).
template <class T>
__device__ __forceinline__ void load_piece(const T *p, T (&v)[8], int h) {
    typedef T vec16 __attribute__((ext_vector_type(16 / sizeof(T))));
    typedef const __attribute__((address_space(1))) vec16 gvec16;
    const vec16 x = *(const gvec16 *)p;
#pragma unroll
    for (int t = 0; t < bcr_per<T>(); ++t) v[h * bcr_per<T>() + t] = x[t];
}


template <class T, int WPB>
struct BcrShared {
    T red[WPB / 2][2 * BCR_NM][BCR_RT + 4];  // partial tiles: [wave pair][n][row]
    T yold[BCR_RT * 2 * BCR_NM];             // outputs read back by subtracting tasks
};

// Chunk table of the block's task (dynamic LDS, sized per launch by the widest task of the
// phase, so short phases keep more blocks resident): per 8-column chunk kc, the position
// of column 8 kc in a member's work vector minus 8 kc, times 2, plus the source (0 = ws,
// 1 = ys); chunks past the padded width repeat the last chunk of the last segment.
extern __shared__ int32_t bcr_tab[];

// Operands of one 32-column step: 8 columns of two M rows and of NNT X columns per lane.
template <class T, int NNT>
struct BcrStep {
    T a0[8], a1[8], b[NNT][8];
};

// Loads of one step; branch-free so that the next step's loads stay in flight while
// the current step's MFMAs run.  Lanes of absent members read the chunk's first member
// (their output columns are never stored).  A piece of X lies in one 8-column
// chunk, whose table entry gives its position in the work vector; the 16 lanes of a lane
// group read 16 adjacent member columns of one chunk, a contiguous run.
template <class T, int NNT>
__device__ __forceinline__ void bcr_fetch_b(BcrStep<T, NNT> &o, const int64_t (&bbase)[NNT], int64_t cs, int k,
                                            const T *wsb, const T *ysb) {
    const int g = (threadIdx.x >> 4) & 3;
#pragma unroll
    for (int h = 0; h < 8 / bcr_per<T>(); ++h) {
        const int c = k + bcr_col<T>(g, h * bcr_per<T>());
        const int32_t e = bcr_tab[c >> 3];
        const T *src = (e & 1) ? ysb : wsb;
        const int64_t pos = wv_pos((int64_t)(e >> 1) + c, cs);  // a piece never crosses a chunk
#pragma unroll
        for (int nt = 0; nt < NNT; ++nt) load_piece(src + bbase[nt] + pos, o.b[nt], h);
    }
}

// One piece of M, read non-temporally: each matrix element is used by one block once per
// application, so it should not evict the member vectors (the X operands, which every
// row tile of a task reads again) from the caches.
template <class T>
__device__ __forceinline__ void load_piece_stream(const T *p, T (&v)[8], int h) {
    typedef T vec16 __attribute__((ext_vector_type(16 / sizeof(T))));
    typedef const __attribute__((address_space(1))) vec16 gvec16;
    const vec16 x = __builtin_nontemporal_load((const gvec16 *)p);
#pragma unroll
    for (int t = 0; t < bcr_per<T>(); ++t) v[h * bcr_per<T>() + t] = x[t];
}

// M operands of one step: the row tile is stored in lane order (see k_repack), so piece
// h of every lane of the wave is one contiguous 64 x 16-byte run.
template <class T>
__device__ __forceinline__ void bcr_fetch_a(const T *A, T (&v)[8]) {
#pragma unroll
    for (int h = 0; h < 8 / bcr_per<T>(); ++h) load_piece_stream(A + h * 64 * bcr_per<T>(), v, h);
}

template <class T, int WPB, int NNT>
__device__ __forceinline__ void bcr_fetch(BcrStep<T, NNT> &o, const BcrShared<T, WPB> &sh,
                                          const int64_t (&bbase)[NNT], int64_t cs, const T *A0, const T *A1,
                                          int k, const T *wsb, const T *ysb) {
    bcr_fetch_a(A0 + (int64_t)BCR_RT * k, o.a0);  // step k / BCR_KS of the row tile
    bcr_fetch_a(A1 + (int64_t)BCR_RT * k, o.a1);
    bcr_fetch_b(o, bbase, cs, k, wsb, ysb);
}

template <class T, int NNT>
__device__ __forceinline__ void bcr_mma(const BcrStep<T, NNT> &o, typename Mfma<T>::v4 (&acc)[2][NNT]) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int nt = 0; nt < NNT; ++nt) {
            acc[0][nt] = Mfma<T>::op(o.a0[j], o.b[nt][j], acc[0][nt]);
            acc[1][nt] = Mfma<T>::op(o.a1[j], o.b[nt][j], acc[1][nt]);
        }
}

template <class T, int WPB, int NNT>
__device__ __forceinline__ void bcr_tile(const BcrTask &tk, BcrShared<T, WPB> &sh, int row0, int mb, int m1,
                                         const int32_t *__restrict__ memb, const int32_t *__restrict__ mask,
                                         T *__restrict__ wsb, T *__restrict__ ysb) {
    using V4 = typename Mfma<T>::v4;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i16 = lane & 15, g = lane >> 4;
    const T *M = static_cast<const T *>(tk.M);
    // M is stored tile by tile in lane order (zero rows pad the last row tile): this
    // lane's values of m tile mt, step k, start at row0 ld + BCR_RT k + 512 mt + P lane
    const T *A0 = M + (int64_t)row0 * tk.ld + bcr_per<T>() * lane;
    const T *A1 = A0 + 16 * BCR_KS;
    // start of this lane's member column (member mi - mbeg of the group, re or im); lanes of
    // absent members read the chunk's first member, whose lines the other lanes fetch anyway
    int64_t bbase[NNT];
#pragma unroll
    for (int nt = 0; nt < NNT; ++nt) {
        const int mi = mb + 8 * nt + (i16 >> 1);
        bbase[nt] = tk.gbase + 16 * (int64_t)((mi < m1 ? mi : mb) - tk.mbeg) + 8 * (i16 & 1);
    }
    V4 acc[2][NNT];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < NNT; ++nt) acc[mt][nt] = V4{0, 0, 0, 0};
    const int kbeg = wave * tk.kq;
    const int nst = max(0, (min(tk.ld, kbeg + tk.kq) - kbeg) / BCR_KS);  // same for the whole wave
    // Latency of the block start: the first step's M operands and the outputs that a
    // subtracting task reads back are requested before the chunk table is copied (the
    // X operands need the table).
    BcrStep<T, NNT> p, q;
    if (nst > 0) {
        bcr_fetch_a(A0 + (int64_t)BCR_RT * kbeg, p.a0);
        bcr_fetch_a(A1 + (int64_t)BCR_RT * kbeg, p.a1);
    }
    // Any active member in this chunk: one flag per lane, the same ballot in every wave,
    // so the whole block leaves together.  It is taken after the first M request, which
    // depends on the task alone, so that the member and mask lookups overlap it.
    const bool on = lane < 8 * NNT && mb + lane < m1 && (!mask || mask[memb[mb + lane]]);
    if (!__ballot(on)) return;
    constexpr int NOUT = BCR_RT * 16 * NNT;
    constexpr int NPT = (NOUT + 64 * WPB - 1) / (64 * WPB);  // outputs per thread
    if (tk.subtract) {
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int o = threadIdx.x + i * 64 * WPB;
            const int n = o / BCR_RT, r = o % BCR_RT;
            const int mi = mb + (n >> 1);
            if (o < NOUT && row0 + r < tk.rows && mi < m1)
                sh.yold[o] = (tk.out_dst ? ysb : wsb)[tk.gbase + 16 * (int64_t)(mi - tk.mbeg) + 8 * (n & 1) +
                                                      wv_pos(tk.out_off + row0 + r, tk.cs)];
        }
    }
    for (int kc = threadIdx.x; kc < (tk.ld >> 3); kc += blockDim.x) bcr_tab[kc] = tk.tab[kc];
    __syncthreads();
    if (nst > 0) {
        // Two operand buffers in turn, two steps per trip with no exit between them: each
        // buffer's loads are then issued a whole MFMA block before their use on every
        // path (with an exit between the halves the compiler sinks the second buffer's
        // loads below the first block).  The prefetch after the last step repeats the
        // last step's addresses; the scheduling barriers keep each prefetch ahead of the
        // MFMAs it overlaps.
        const int klast = kbeg + (nst - 1) * BCR_KS;
        bcr_fetch_b(p, bbase, tk.cs, kbeg, wsb, ysb);
        int st = 0;
        for (; st + 2 <= nst; st += 2) {
            bcr_fetch<T, WPB, NNT>(q, sh, bbase, tk.cs, A0, A1, kbeg + (st + 1) * BCR_KS, wsb, ysb);
            __builtin_amdgcn_sched_barrier(0);
            bcr_mma(p, acc);
            bcr_fetch<T, WPB, NNT>(p, sh, bbase, tk.cs, A0, A1, min(kbeg + (st + 2) * BCR_KS, klast), wsb, ysb);
            __builtin_amdgcn_sched_barrier(0);
            bcr_mma(q, acc);
        }
        if (st < nst) bcr_mma(p, acc);
    }
    // Sum of the waves' partial tiles in a fixed order: the upper half of the waves
    // store, the lower half adds and stores, then every thread sums the WPB/2 slots.
    // Accumulator v of lane (i16, g) is row Mfma::row(g, v) of m tile mt, column i16
    // of n tile nt.
    constexpr int H = WPB / 2;
    if (wave >= H) {
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < NNT; ++nt)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    sh.red[wave - H][16 * nt + i16][16 * mt + Mfma<T>::row(g, v)] = acc[mt][nt][v];
    }
    __syncthreads();
    if (wave < H) {
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < NNT; ++nt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    T &slot = sh.red[wave][16 * nt + i16][16 * mt + Mfma<T>::row(g, v)];
                    slot = acc[mt][nt][v] + slot;
                }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
        const int o = threadIdx.x + i * 64 * WPB;
        const int n = o / BCR_RT, r = o % BCR_RT;
        const int mi = mb + (n >> 1);
        if (o >= NOUT || row0 + r >= tk.rows || mi >= m1) continue;
        if (mask && !mask[memb[mi]]) continue;
        T v = 0;
#pragma unroll
        for (int w = 0; w < H; ++w) v += sh.red[w][n][r];
        T *y = (tk.out_dst ? ysb : wsb) + tk.gbase + 16 * (int64_t)(mi - tk.mbeg) + 8 * (n & 1) +
               wv_pos(tk.out_off + row0 + r, tk.cs);
        *y = tk.subtract ? sh.yold[o] - v : v;
    }
}

// waves per SIMD asked of the register allocator (f32: 4, i.e. at most 128 VGPRs)
template <class T> struct BcrOcc { static constexpr int v = 4; };
template <> struct BcrOcc<double> { static constexpr int v = 2; };

template <class T, int WPB>
__global__ void __launch_bounds__(64 * WPB, BcrOcc<T>::v) k_bcr_mfma(const BcrTask *__restrict__ tasks,
                                                       const int32_t *__restrict__ blkoff, int ntasks,
                                                       const int32_t *__restrict__ memb,
                                                       const int32_t *__restrict__ mask, T *__restrict__ wsb,
                                                       T *__restrict__ ysb) {
    __shared__ BcrShared<T, WPB> sh;
    // Workgroups are dealt to the 8 XCDs round-robin; renumber them so that the row
    // tiles of one task (which read the same input vectors) run on the same XCD and
    // share its L2.
    const int nb = gridDim.x, b = blockIdx.x;
    const int q = nb >> 3, rem = nb & 7, x = b & 7, i = b >> 3;
    const int lb = x < rem ? x * (q + 1) + i : rem * (q + 1) + (x - rem) * q + i;
    const int t = find_sys2(blkoff, ntasks, lb);
    const BcrTask &tk = tasks[t];
    const int local = lb - blkoff[t];
    const int rt = local / tk.nmc, mchunk = local - rt * tk.nmc;
    const int m1 = tk.mend;
    const int mb = tk.mbeg + mchunk * 8 * tk.nnt;
    if (tk.nnt == 1)
        bcr_tile<T, WPB, 1>(tk, sh, rt * BCR_RT, mb, m1, memb, mask, wsb, ysb);
    else
        bcr_tile<T, WPB, 2>(tk, sh, rt * BCR_RT, mb, m1, memb, mask, wsb, ysb);
}

// Value of DoF g of system d's output: ys[pos(g)] on skeleton DoFs; interiors:
// x_i = Kii^{-1} r_i - F^T x_e (r: the system's input, ys: its skeleton solution column).
template <class T>
__device__ __forceinline__ typename P2<T>::t cond_bwd_value(const PrecDesc &d, int64_t g, const T *__restrict__ r_s,
                                                            const T *__restrict__ ys) {
    using T2 = typename P2<T>::t;
    if (g < d.cell_off) {
        const T *yp = ys + wv_pos(d.dof_pos[g], d.cs);
        return T2{yp[0], yp[8]};
    }
    const T2 *r = reinterpret_cast<const T2 *>(r_s);
    const int gi = (int)(g - d.cell_off);
    const int64_t c = gi / d.n_int;
    const int m = gi - (int)c * d.n_int;
    const T *Ki = reinterpret_cast<const T *>(d.kiinv) + c * d.n_int * d.n_int + m;  // transposed: [c][q][m]
    const T2 *ri = r + d.cell_off + c * d.n_int;
    T2 acc{0, 0};
#pragma unroll 4
    for (int q = 0; q < d.n_int; ++q) {
        acc.x += Ki[q * d.n_int] * ri[q].x;
        acc.y += Ki[q * d.n_int] * ri[q].y;
    }
    const T *F = reinterpret_cast<const T *>(d.F) + c * d.ne * d.n_int;
    const int32_t *cp = d.cell_pos + c * d.ne;
#pragma unroll 4
    for (int le = 0; le < d.ne; ++le) {
        const T f = F[le * d.n_int + m];
        const T *yp = ys + wv_pos(cp[le], d.cs);
        acc.x -= f * yp[0];
        acc.y -= f * yp[8];
    }
    return acc;
}

// x = the output of every system (one block per 256 DoFs of one system).
template <class T>
__global__ void __launch_bounds__(256) k_cond_bwd(const PrecDesc *__restrict__ pd, const int64_t *__restrict__ off,
                                                  const int64_t *__restrict__ soff, const int32_t *__restrict__ blkoff,
                                                  int ns, const int32_t *__restrict__ mask, const T *__restrict__ rb,
                                                  const T *__restrict__ ysb, T *__restrict__ xb) {
    using T2 = typename P2<T>::t;
    const int s = find_sys2(blkoff, ns, blockIdx.x);
    if (mask && !mask[s]) return;
    const PrecDesc &d = pd[s];
    const int64_t g = (int64_t)(blockIdx.x - blkoff[s]) * 256 + threadIdx.x;
    if (g >= d.n) return;
    reinterpret_cast<T2 *>(xb + off[s])[g] = cond_bwd_value<T>(d, g, rb + off[s], ysb + soff[s]);
}

// The same outputs written only to the member-interleaved copy of the grouped SpMV (see
// SpmvGroup::xoff).  A block takes IL_TILE consecutive DoFs of every member of one group:
// wave k computes the tile's DoFs of member k (the reads of k_cond_bwd), the tile is
// transposed through LDS, and the block writes it as one contiguous run of the copy.
// Padding slots (member index >= nm) and masked members receive zeros, so that every
// write covers whole lines (the grouped SpMV ignores those members' results); a block
// whose group has no active member returns at once.
// blkoff: schedule of ceil(rows / IL_TILE) blocks per group; 64 SPMV_GMAX threads per block.
template <class T>
__global__ void __launch_bounds__(64 * SPMV_GMAX) k_cond_bwd_il(const PrecDesc *__restrict__ pd,
                                                                const int64_t *__restrict__ off,
                                                                const int64_t *__restrict__ soff,
                                                                const SpmvGroup *__restrict__ groups,
                                                                const int32_t *__restrict__ blkoff, int ng,
                                                                const int32_t *__restrict__ mask,
                                                                const T *__restrict__ rb, const T *__restrict__ ysb,
                                                                T *__restrict__ xib) {
    static_assert(IL_TILE == 64, "one wave per member and tile");
    using T2 = typename P2<T>::t;
    constexpr int LD = SPMV_GMAX + 1;  // LDS row stride (entries): spreads a wave's stores over the banks
    __shared__ T2 tile[IL_TILE * LD];
    const int gi = find_sys2(blkoff, ng, blockIdx.x);
    const SpmvGroup &G = groups[gi];
    const int npad = G.npad, nm = G.nm;
    const int64_t n = pd[G.rep].n;  // members share K, hence the DoF count
    const int64_t g0 = (int64_t)(blockIdx.x - blkoff[gi]) * IL_TILE;
    if (mask && !__syncthreads_or((int)threadIdx.x < nm && mask[G.mem[threadIdx.x]])) return;
    const int lane = (int)threadIdx.x & 63;
    // the wave's member: uniform over the wave, so its descriptor loads stay scalar
    const int k = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    if (k < npad) {
        const int64_t g = g0 + lane;
        T2 v{0, 0};
        if (k < nm) {
            const int s = G.mem[k];
            if ((!mask || mask[s]) && g < n) v = cond_bwd_value<T>(pd[s], g, rb + off[s], ysb + soff[s]);
        }
        tile[lane * LD + k] = v;
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t >= IL_TILE * npad) return;
    const int l = t / npad, kk = t - l * npad;
    if (g0 + l >= n) return;
    (reinterpret_cast<T2 *>(xib) + G.xoff + g0 * npad)[t] = tile[l * LD + kk];
}

template <class T>
void launch_bcr_phases(const PrecBatch &P, const int32_t *mask, T *ws, T *ys, hipStream_t st) {
    constexpr int prec = sizeof(T) == 8 ? 0 : 1;
    for (const PrecPhase &ph : P.phases) {
        const int nb = ph.sched[prec].nblocks;
        if (!nb) continue;
        k_bcr_mfma<T, BCR_WPB><<<nb, 64 * BCR_WPB, sizeof(int32_t) * (ph.max_ld / 8), st>>>(
            ph.tasks[prec].p, ph.sched[prec].blkoff.p, ph.ntasks, P.memb.p, mask, ws, ys);
    }
    THM_HIP(hipGetLastError());
}
template void launch_bcr_phases<double>(const PrecBatch &, const int32_t *, double *, double *, hipStream_t);
template void launch_bcr_phases<float>(const PrecBatch &, const int32_t *, float *, float *, hipStream_t);

// ------------------------------------------------------------------ batched transpose (setup)
__global__ void __launch_bounds__(256) k_batch_transpose(int64_t total, int rows, int cols,
                                                         const double *__restrict__ src, double *__restrict__ dst) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= total) return;
    const int64_t per = (int64_t)rows * cols, b = e / per;
    const int rem = (int)(e - b * per), i = rem / cols, j = rem - i * cols;
    dst[b * per + (int64_t)j * rows + i] = src[e];
}

void launch_batch_transpose(int64_t count, int rows, int cols, const double *src, double *dst, hipStream_t st) {
    const int64_t total = count * rows * cols;
    if (total <= 0) return;
    k_batch_transpose<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(total, rows, cols, src, dst);
    THM_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ padded copies (setup)
// Element (r, c) of the padded apply matrix (zero outside the true rows and segments).
__device__ double repack_value(const RepackDesc &d, int64_t r, int pc) {
    if (r >= d.rows) return 0.0;
    for (int q = 0; q < d.nseg; ++q) {
        const int j = pc - d.seg_pstart[q];
        if (j >= 0 && j < d.seg_len[q]) return d.src[r * d.cols + d.seg_col[q] + j];
    }
    return 0.0;
}

// Row and column of slot w of a BCR_RT x BCR_KS tile stored in lane order for values of
// P per 16-byte piece: m tile mt = w / 512, then piece h, lane L = i16 + 16 g, value t,
// holding row 16 mt + i16 and step column bcr_col(g, h P + t).
template <class T>
__device__ void repack_slot(int w, int &r, int &c) {
    constexpr int P = bcr_per<T>();
    const int mt = w / 512, w2 = w % 512;
    const int h = w2 / (64 * P), L = (w2 % (64 * P)) / P, t = w2 % P;
    r = 16 * mt + L % 16;
    c = bcr_col<T>(L / 16, h * P + t);
}

// Copy of the apply matrices in the layout the MFMA apply streams: rows rounded up to
// BCR_RT, the columns of each segment at its padded start, cut into BCR_RT x BCR_KS
// tiles stored one after another along a row tile, each tile in lane order.  A wave's
// operand loads of one step are then contiguous runs, and its column range one stream.
__global__ void __launch_bounds__(256) k_repack(const RepackDesc *__restrict__ ds, const int32_t *__restrict__ blkoff,
                                                int nd, double *__restrict__ dst64, float *__restrict__ dst32) {
    const int di = find_sys2(blkoff, nd, blockIdx.x);
    const RepackDesc &d = ds[di];
    const int64_t e = (int64_t)(blockIdx.x - blkoff[di]) * 256 + threadIdx.x;
    const int64_t prows = (int64_t)(d.rows + BCR_RT - 1) / BCR_RT * BCR_RT;
    if (e >= prows * d.ld) return;
    constexpr int TS = BCR_RT * BCR_KS;
    const int64_t tile = e / TS;
    const int w = (int)(e - tile * TS);
    const int nk = d.ld / BCR_KS;
    const int64_t rt = tile / nk;
    const int kc = (int)(tile - rt * nk);
    int r, c;
    repack_slot<double>(w, r, c);
    dst64[d.poff + e] = repack_value(d, rt * BCR_RT + r, kc * BCR_KS + c);
    repack_slot<float>(w, r, c);
    dst32[d.poff + e] = (float)repack_value(d, rt * BCR_RT + r, kc * BCR_KS + c);
}

void launch_repack(const std::vector<RepackDesc> &d, double *dst64, float *dst32, hipStream_t st) {
    if (d.empty()) return;
    std::vector<int64_t> units(d.size());
    for (size_t i = 0; i < d.size(); ++i) units[i] = (int64_t)(d[i].rows + BCR_RT - 1) / BCR_RT * BCR_RT * d[i].ld;
    Sched sc;
    sc.build(units, 256, st);
    DBuf<RepackDesc> dd;
    dd.upload(d, st);
    if (sc.nblocks) k_repack<<<sc.nblocks, 256, 0, st>>>(dd.p, sc.blkoff.p, (int)d.size(), dst64, dst32);
    THM_HIP(hipGetLastError());
    THM_HIP(hipStreamSynchronize(st));
}

template <class T>
void launch_prec_apply(const PrecBatch &P, const PrecDesc *d, const int64_t *off, int ns, const int32_t *mask,
                       const T *r, T *x, T *ws, T *ys, T *tw, hipStream_t st, const IlOut<T> *il) {
    if (P.cfr.nblocks) k_cond_fr<T><<<P.cfr.nblocks, 256, 0, st>>>(d, off, P.toff.p, P.cfr.blkoff.p, ns, mask, r, tw);
    if (P.skel.nblocks)
        k_cond_fwd<T><<<P.skel.nblocks, 256, 0, st>>>(d, off, P.soff.p, P.toff.p, P.skel.blkoff.p, ns, mask, r, tw, ws);
    launch_bcr_phases<T>(P, mask, ws, ys, st);
    if (il) {
        if (il->sched->nblocks)
            k_cond_bwd_il<T><<<il->sched->nblocks, 64 * SPMV_GMAX, 0, st>>>(d, off, P.soff.p, il->groups, il->sched->blkoff.p,
                                                                 il->ng, mask, r, ys, il->xi);
    } else if (P.dofs.nblocks) {
        k_cond_bwd<T><<<P.dofs.nblocks, 256, 0, st>>>(d, off, P.soff.p, P.dofs.blkoff.p, ns, mask, r, ys, x);
    }
    THM_HIP(hipGetLastError());
}

template void launch_prec_apply<double>(const PrecBatch &, const PrecDesc *, const int64_t *, int, const int32_t *,
                                        const double *, double *, double *, double *, double *, hipStream_t,
                                        const IlOut<double> *);
template void launch_prec_apply<float>(const PrecBatch &, const PrecDesc *, const int64_t *, int, const int32_t *,
                                       const float *, float *, float *, float *, float *, hipStream_t,
                                       const IlOut<float> *);


}  // namespace thm
