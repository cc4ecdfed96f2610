// Device descriptors and kernel launchers shared by the HIP sources.
#pragma once
#include <map>

#include "thm_internal.h"

namespace thm {

constexpr int VCHUNK = 4096;  // scalars per block in Krylov vector kernels (even)
constexpr int NPW = 4;        // partial-sum slots per block (one per wave)

struct MatDesc {
    int64_t n;
    const int32_t *rowptr, *col;
    const void *kval;
    const int32_t *crowptr, *ccol;
    const void *cval;
    // K in SELL-64 (rows sorted by length within windows of SELL_SIGMA, slices of 64,
    // entries column-major within a slice, padded to the slice's longest row with zero
    // values): the same values as kval
    const int32_t *sl_ptr, *sl_col;  // entry offset of each slice (n_slices + 1); columns
    const int32_t *sl_row;           // original row of each slice lane (-1: none)
    const void *sl_val;
};
constexpr int SELL_C = 64;        // rows per slice (one wave, one row per lane)
constexpr int SELL_SIGMA = 1024;  // sorting window (rows)
constexpr int SPMV_SELL = 19;     // SpMV variant code of the SELL-64 kernel (256 rows per block)
// Grouped SELL-64 (variant code SPMV_SELL_GROUP): systems of a batch with the same K share
// one read of it per product.  A group holds at most SPMV_GMAX systems.
constexpr int SPMV_SELL_GROUP = 20;
// The grouped product reading x from the member-interleaved copy that the preconditioner
// writes in an Arnoldi step (chosen explicitly; elsewhere the batch uses SPMV_SELL_GROUP).
constexpr int SPMV_SELL_GROUP_IL = 29;
constexpr int SPMV_GMAX = 16;
struct SpmvGroup {
    int32_t rep;                 // system whose SELL arrays hold the shared K
    int32_t nm;                  // member systems (1 .. SPMV_GMAX)
    int32_t npad;                // nm rounded up to 4, 8, 12 or 16 (npad / 4 waves per slice)
    int32_t mem[SPMV_GMAX];      // member system indices
    const uint8_t *crow;         // per row of K: 1 if some member's C row has entries
    // member-interleaved copy of the group's vectors (complex entries): member j's value at row r
    // lies at xoff + r npad + j, so one row of K meets every member's value in one contiguous run
    int64_t xoff;
};
// Host: SELL-64 layout of a CSR pattern; src[e] = CSR index of entry e, or -1 (padding).
void sell_build(int64_t n, const std::vector<int32_t> &rowptr, const std::vector<int32_t> &col,
                std::vector<int32_t> &ptr, std::vector<int32_t> &scol, std::vector<int32_t> &src,
                std::vector<int32_t> &row);
// Device: SELL values from the CSR values (FP64 and FP32 copies).
void launch_sell_fill(int64_t ne, const int32_t *src, const double *kval, double *v64, float *v32, hipStream_t st);

// Flattened block schedule: block b belongs to system s with blkoff[s] <= b < blkoff[s+1].
// The device array holds blkoff[0..ns] followed by the block -> system map, so a kernel
// finds its system with one load: blkoff[ns + 1 + b].
struct Sched {
    DBuf<int32_t> blkoff;
    std::vector<int32_t> h;
    int nblocks = 0;
    void build(const std::vector<int64_t> &units, int64_t per_block, hipStream_t st) {
        const size_t ns = units.size();
        h.assign(ns + 1, 0);
        for (size_t s = 0; s < ns; ++s) h[s + 1] = h[s] + (int32_t)((units[s] + per_block - 1) / per_block);
        nblocks = h.back();
        std::vector<int32_t> all(h);
        all.reserve(ns + 1 + nblocks);
        for (size_t s = 0; s < ns; ++s)
            for (int32_t b = h[s]; b < h[s + 1]; ++b) all.push_back((int32_t)s);
        blkoff.upload(all, st);
    }
};

// A batch of independent systems sharing kernel launches.
struct Batch {
    int ns = 0;
    int maxcols = 64;                  // columns of the partial-sum buffer (>= 2 (restart + 1))
    DBuf<int64_t> off, len, nvec;      // scalar offset, scalar length (2n), complex length n
    std::vector<int64_t> h_off, h_len, h_nvec;
    int64_t Ltot = 0;                  // scalars per vector slot
    Sched vs;                          // VCHUNK scalars per block
    Sched es;                          // 256 complex entries per block
    std::map<int, Sched> spmv;         // per SpMV variant (10 * lanes_per_row + unroll): 256 / lpr rows per block
    void init(const std::vector<int64_t> &n, int maxcols_, hipStream_t st) {
        ns = (int)n.size();
        maxcols = maxcols_;
        h_off.assign(ns, 0);
        h_len.assign(ns, 0);
        h_nvec = n;
        int64_t o = 0;
        for (int s = 0; s < ns; ++s) {
            h_off[s] = o;
            h_len[s] = 2 * n[s];
            o += 2 * n[s];
            o = (o + 63) & ~int64_t(63);  // 512-byte aligned slots per system
        }
        Ltot = o;
        off.upload(h_off, st);
        len.upload(h_len, st);
        nvec.upload(h_nvec, st);
        vs.build(h_len, VCHUNK, st);
        es.build(h_nvec, 256, st);
    }
    const Sched &spmv_sched(int lpr, hipStream_t st) {
        auto it = spmv.find(lpr);
        if (it != spmv.end()) return it->second;
        Sched &sc = spmv[lpr];
        sc.build(h_nvec, 256 / (lpr / 10), st);
        return sc;
    }
};

// ---- SpMV and Krylov vector kernels (kernels_la.hip)
template <class T>
void launch_spmv(int lpr, const MatDesc *mats, const int64_t *off, const Sched &sc, int ns, const int32_t *mask,
                 const T *x, T *y, const T *b, float csign, hipStream_t st);
// Grouped SELL-64 product over the groups of a batch (schedule: one unit per wave, i.e.
// slices of the representative times npad / 4, four units per block); same arguments as
// launch_spmv otherwise.
template <class T>
void launch_spmv_group(const MatDesc *mats, const int64_t *off, const SpmvGroup *groups, const Sched &sc, int ng,
                       const int32_t *mask, const T *x, T *y, const T *b, float csign, hipStream_t st);
// The same product with x read from the member-interleaved copy xi (see SpmvGroup::xoff):
// the same sums in the same order, so the same bits.
template <class T>
void launch_spmv_group_i(const MatDesc *mats, const int64_t *off, const SpmvGroup *groups, const Sched &sc, int ng,
                         const int32_t *mask, const T *xi, T *y, float csign, hipStream_t st);
template <class T>
void launch_dots(const Batch &B, const int32_t *mask, const int32_t *jcnt, const T *V, int64_t ld, const T *w,
                 double *part, int cplx, hipStream_t st);
template <class T>
void launch_cgs_update(const Batch &B, const int32_t *mask, const int32_t *jcnt, const T *V, int64_t ld, T *w,
                       const double *h, int ldh, double *part, hipStream_t st);
template <class T>
void launch_norm2(const Batch &B, const int32_t *mask, const T *x, double *part, hipStream_t st);
template <class TI, class TO>
void launch_scale(const Batch &B, const int32_t *mask, const double *scal, int invert, const TI *x, TO *y1,
                  const int32_t *jcol, int64_t ld1, TO *y2, hipStream_t st, int32_t *step_ctr = nullptr);
template <class T>
void launch_lincomb(const Batch &B, const int32_t *mask, const int32_t *kcnt, const T *V, int64_t ld,
                    const double *coef, int ldc, T *y, hipStream_t st);
template <class TX, class TZ>
void launch_axpy(const Batch &B, const int32_t *mask, const double *scal, const TZ *z, TX *x, hipStream_t st);
void launch_norm_finish(const Batch &B, const double *part, const int32_t *mask, double *out, const double *bnorm,
                        double rtol, double *resid, int32_t *running, hipStream_t st);
void launch_reduce_cols(const Batch &B, const int32_t *mask, const int32_t *jcnt, int ncols_fixed,
                        const double *part, double *out, int ldo, int accumulate, hipStream_t st);
// Start of a cycle: tolerance read from rtol_d; resets *step_ctr (if non-null); writes each
// system's running flag to hrun (host-visible, may be null).
void launch_cycle_start(const Batch &B, const double *part, int32_t *running, int32_t *active, int32_t *jcnt,
                        const double *bnorm, const double *rtol_d, double *g, int m, double *beta, double *resid,
                        int32_t *iters, int max_iter, int32_t *step_ctr, int32_t *hrun, hipStream_t st);
// End of an Arnoldi step: the flags go to host slot (step / spc) mod nslots.
void launch_arnoldi_finish(const Batch &B, const double *part, int32_t *active, int32_t *jcnt, const double *hcol,
                           int ldh, double *H, double *cs, double *sn, double *g, double *hnext,
                           const double *bnorm, const double *rtol_d, int m, int32_t *iters, int max_iter,
                           double *est, int32_t *hflags, const int32_t *step_ctr, int spc, int nslots,
                           hipStream_t st);
void launch_hsolve(const Batch &B, const int32_t *running, const int32_t *jcnt, const double *H, const double *g,
                   double *y, int m, hipStream_t st);
template <class T>
void launch_zero_flagged(const Batch &B, const uint8_t *const *dirs, T *x, hipStream_t st);

// ---- preconditioner (kernels_prec.hip)
// Per-system preconditioner description for batched application.
// Skeleton work vectors of the apply (ws, ys): the members of a factor group share one
// region of 8-position chunks.  Chunk q holds, for every padded member column of the group
// (member j: real part in column 2j, imaginary part in column 2j + 1), its values at positions
// 8q .. 8q + 7, so a chunk is cs = 16 x (padded members) scalars.  A member column's value at
// position p lies wv_pos(p, cs) after the column's start, and the imaginary column starts 8
// after the real one.
__host__ __device__ inline int64_t wv_pos(int64_t p, int64_t cs) { return (p >> 3) * cs + (p & 7); }

struct PrecDesc {
    int64_t n;                 // complex DoFs
    int64_t n_skel;            // skeleton DoFs
    int64_t cell_off;          // first interior DoF
    int64_t sp;                // padded skeleton length (positions 0 .. sp - 1, a multiple of 8)
    int64_t cs;                // chunk stride of the system's factor group (see wv_pos)
    int32_t n_cells, n_loc, n_int, ne, nlayers;
    const int32_t *cell_dofs;  // n_cells * n_loc
    const int32_t *skel_dof;   // skeleton position -> global DoF
    const int32_t *skel_pos;   // skeleton position -> padded position in the work vectors
    const int32_t *dof_pos;    // global DoF -> padded position (-1: interior)
    const int32_t *cell_pos;   // n_cells * ne: padded positions of each cell's skeleton DoFs
    const int32_t *cond_ptr, *cond_cell, *cond_loc;
    // double or float: per cell K_ii^{-1} stored transposed ([c][q][m] = (K_ii^{-1})_{mq}),
    // F_c = K'_ei K_ii^{-1} ([c][le][m]) and its transpose ([c][m][le]); the transposed
    // layouts make the reads of one cell's threads consecutive
    const void *kiinv, *F, *FT;
};

// One dense task of the cyclic-reduction application (see kernels_prec.hip): the
// product of a rows x (padded) matrix with the concatenated input segments of every
// member of a factor group.  Columns of segment q occupy [seg_pstart[q], seg_pstart[q+1]);
// the part past the layer's true width is zero in the matrix and in the vectors.
constexpr int SEGMAX = 16;   // input segments of one task (the dense last block reads all its positions)
constexpr int BCR_KS = 32;   // columns per MFMA step (4 lane groups x 8 consecutive columns)
constexpr int BCR_RT = 32;   // rows per block (two 16-row MFMA tiles)
constexpr int BCR_NM = 16;   // members per block at most (two 16-wide n tiles, re and im columns)
constexpr int BCR_TAB = 4096;  // 8-column chunks of one task row at most (32768 padded columns)
struct BcrTask {
    const void *M;             // row-major rows x ld (double or float), 16-byte aligned rows
    int32_t rows, ld, nseg, group;
    int32_t mbeg, mend;        // the group's members: PrecBatch::memb[mbeg, mend)
    int32_t kq;                // columns per wave (multiple of BCR_KS)
    int32_t nnt;               // 16-wide n tiles per block (1 or 2): members per block = 8 nnt
    int32_t nmc;               // member chunks of the group
    int32_t out_dst, subtract;
    int32_t seg_pstart[SEGMAX + 1];
    int32_t seg_src[SEGMAX];   // 0 = ws (reduced RHS), 1 = ys (solution)
    int64_t seg_off[SEGMAX];   // padded position of the segment in a member's work vector
    int64_t out_off;           // padded position of the output block
    int64_t gbase;             // start of the group's region in the work vectors
    int64_t cs;                // its chunk stride (see wv_pos)
    // per 8-column chunk kc (ld / 8 entries): 2 (p - 8 kc) + src, where p is the position
    // of column 8 kc in a member's work vector and src selects ws (0) or ys (1); chunks
    // past the padded width repeat the last chunk of the last segment (zero in M)
    const int32_t *tab;
};
// chunk table entries of one task (host side, see BcrTask::tab)
void bcr_chunk_table(const BcrTask &t, std::vector<int32_t> &out);
constexpr int BCR_WPB = 4;   // waves per block: the column split of a row tile

// Copy of one apply matrix into the padded layout (setup only).
struct RepackDesc {
    const double *src;         // rows x cols, row-major
    int32_t rows, cols, ld, nseg;
    int64_t poff;              // destination offset
    int32_t seg_col[SEGMAX], seg_len[SEGMAX], seg_pstart[SEGMAX];
};
void launch_repack(const std::vector<RepackDesc> &d, double *dst64, float *dst32, hipStream_t st);
// dst[b] = src[b]^T for count row-major rows x cols matrices (setup only)
void launch_batch_transpose(int64_t count, int rows, int cols, const double *src, double *dst, hipStream_t st);

struct PrecPhase {
    DBuf<BcrTask> tasks[2];    // FP64, FP32 matrices
    DBuf<int32_t> tab;         // chunk tables of the tasks
    int max_ld = 0;            // widest task (padded columns)
    Sched sched[2];            // blocks = row blocks x member chunks
    int ntasks = 0;
};

struct PrecBatch {
    int ns = 0;
    DBuf<PrecDesc> d64, d32;
    DBuf<int64_t> soff;            // start of each system's real column (group start + 16 j)
    int64_t Stot = 0;              // scalars per skeleton slot
    Sched skel;                    // 256 skeleton entries per block
    Sched dofs;                    // 256 DoFs per block
    Sched cfr;                     // 256 (cell, skeleton local DoF) pairs per block
    DBuf<int64_t> toff;            // complex offset of each system's per-cell condensation terms
    int64_t Ttot = 0;              // complex entries of all condensation terms
    DBuf<int32_t> memb_ptr, memb;  // factor group -> member systems
    std::vector<PrecPhase> phases; // forward levels, top, backward levels
};

template <class T>
void launch_bcr_phases(const PrecBatch &P, const int32_t *mask, T *ws, T *ys, hipStream_t st);
// x = diag(K, K)^{-1} r for every system of the batch; ws, ys: skeleton work vectors
// (PrecBatch::Stot scalars), tw: condensation terms (2 PrecBatch::Ttot scalars).
// Output in the member-interleaved layout of the grouped SpMV instead of the systems' own
// vectors: the SpMV groups, a schedule of IL_TILE DoFs of a group per block, the copy.
constexpr int IL_TILE = 64;
template <class T>
struct IlOut {
    const SpmvGroup *groups;
    const Sched *sched;
    int ng;
    T *xi;
};
template <class T>
void launch_prec_apply(const PrecBatch &P, const PrecDesc *d, const int64_t *off, int ns, const int32_t *mask,
                       const T *r, T *x, T *ws, T *ys, T *tw, hipStream_t st, const IlOut<T> *il = nullptr);

// ---- complete inverse (K + iC)^{-1} through K^{-1} and a boundary correction (kernels_full.hip)
struct FullDesc {
    int maxr = 0, nchmax = 0;        // largest boundary size; column chunks of M^{-1} per row
    const int64_t *goff = nullptr;   // ns + 1: system s owns Gamma entries [goff[s], goff[s + 1])
    const int32_t *gam = nullptr;    // boundary DoFs (complex index within the system)
    const int32_t *cptr = nullptr;   // C_G rows: entries [cptr[g], cptr[g + 1]) of row g (absolute)
    const int32_t *ccol = nullptr;   // Gamma-local columns of C_G
    const void *cval64 = nullptr, *cval32 = nullptr;
    const int64_t *moff = nullptr;   // complex offset of the system's M^{-1} (shared by identical systems)
    const void *m64 = nullptr, *m32 = nullptr;  // M^{-1}, complex column-major
};
// Setup of S_G: unit vectors at Gamma entries 2k, 2k + 1 and the gather of the matching
// columns of K^{-1}; k = k0 + kadd[s] per system (kadd null: k0).
void launch_full_unit(const FullDesc &F, int ns, const int32_t *mask, const int64_t *off, const int32_t *kadd,
                      int k0, double val, double *x, hipStream_t st);
void launch_full_gather(const FullDesc &F, int ns, const int32_t *mask, const int64_t *off, const int32_t *kadd,
                        int k0, const double *z, const int64_t *soff, double *S, hipStream_t st);
void launch_full_block(int r, const double *S, const int32_t *cptr, const int32_t *ccol, const double *cval,
                       double *Bm, hipStream_t st);
void launch_full_extract(int r, const double *Inv, double *M64, float *M32, hipStream_t st);
// w[Gamma] = M^{-1} ((+-i) C_G z_G) (w zero elsewhere); u, part: scratch
template <class T>
void launch_full_correct(const FullDesc &F, int ns, const int32_t *mask, const int64_t *off, int conj, const T *z,
                         T *u, T *part, T *w, hipStream_t st);

// Setup (FP64): condensation, dense block assembly, block LU with explicit inverses.
void launch_condense(int ncells, int n_loc, int n_int, const double *Kel, const int32_t *cell_dofs,
                     const uint8_t *dir, double *kiinv, double *F, double *Kcond, int32_t *status,
                     hipStream_t st);
void launch_fill(double *p, int64_t n, double v, hipStream_t st);
void launch_tgt_gather(int64_t ntgt, const int64_t *tgt_index, const int32_t *tgt_kind, const int32_t *tgt_ptr,
                       const int32_t *tgt_src, const double *Kcond, double *sinv, double *lf, hipStream_t st);
void launch_dir_identity(int64_t n_skel, const int32_t *skel_dof, const uint8_t *dir, const int64_t *boff,
                         const int64_t *sinv_off, const int32_t *bsize, int nlayers, double *sinv, hipStream_t st);

struct GemmDesc {
    int m, n, k;               // C (m x n) = alpha op(A) op(B) + beta C
    int ta, tb;                // 1: operand stored transposed
    const double *A, *B;
    double *C;
    int lda, ldb, ldc;
    double alpha, beta;
};
void launch_gemm_batched(const std::vector<GemmDesc> &g, hipStream_t st, DBuf<GemmDesc> &scratch,
                         Sched &sched);

struct InvDesc {
    int n;
    double *A, *W;             // input A (n x n, overwritten); W is scratch (n x n)
    double *out;               // final inverse (n x n, leading dimension ldo)
    int32_t *piv;              // 2n: pivot rows, then the column permutation
    int ldo;
};
// Batched Gauss-Jordan inversion with partial pivoting in panels of 64 columns and rank-64
// product updates (kernels_inv.hip); status |= 1 for a zero or non-finite pivot.
void launch_invert_blocked(const std::vector<InvDesc> &d, int32_t *status, hipStream_t st);
// At (n x m, leading dimension ldt) = alpha * A^T, A (m x n, leading dimension lda)
void launch_transpose(const double *A, int m, int n, int lda, double *At, int ldt, double alpha, hipStream_t st);
void launch_compare(const void *a, const void *b, int64_t n8, int32_t *mismatch, hipStream_t st);
void launch_convert(const double *a, float *b, int64_t n, hipStream_t st);

// ---- finite elements (kernels_fe.hip)
struct FeTables {
    int npts = 0;
    DBuf<double> pts, w;         // npts x 3, npts
    DBuf<double> val, curl;      // n_loc x 3 x npts
    DBuf<double> ref;            // reference mass and curl-curl matrices of the cell (2 n_loc^2; set on first use)
};
void fe_gauss(int q, DBuf<double> &x, DBuf<double> &w, hipStream_t st);
void fe_tables_cell(int dim, int p, int q, const LocalFn *fns_dev, int n_loc, FeTables &T, hipStream_t st);
void fe_tables_side(int dim, int p, int q, int axis, int side, const LocalFn *fns_dev, int n_loc, FeTables &T,
                    hipStream_t st);
void launch_element_matrices(int dim, int64_t ncells, int n_loc, FeTables &T, const double *h,
                             const double *mu, const double *eps, double omega, double *Kel, hipStream_t st);
void launch_gather(int64_t nnz, const int32_t *gptr, const int32_t *gsrc, const double *src, double scale,
                   double *val, hipStream_t st);
void launch_side_mass(int dim, int nsides, const int32_t *side_axis, const int32_t *side_side,
                      const int32_t *side_fn, int nf, int n_loc, const FeTables *tabs_dev_host[6],
                      const double *h, double *out, hipStream_t st);
// Interface sides of a DDM subdomain with a transmission factor s (see thm_problem.transmission):
// scale the side blocks selected by the bit mask sel (bit 2 axis + side), and add a multiple of
// side blocks [s0, s1) of one (axis, side) group into the element matrices of their cells.
void launch_side_scale(int nsides, const int32_t *side_axis, const int32_t *side_side, uint32_t sel, int nf,
                       double f, const double *in, double *out, hipStream_t st);
void launch_side_to_elem(int s0, int s1, const int32_t *side_cell, const int32_t *side_axis,
                         const int32_t *side_side, const int32_t *side_fn, int nf, int n_loc, double coef,
                         const double *blk, double *kel, hipStream_t st);
void launch_side_load(int dim, int nsides, const int32_t *side_cell, const int32_t *side_axis,
                      const int32_t *side_side, const int32_t *side_fn, int nf, int n_loc,
                      const FeTables *tabs[6], const double *h, const double *lo, const int32_t *ncell3,
                      const double *dirv, const double *pol_re, const double *pol_im, double omega,
                      double *out, hipStream_t st);
void launch_gather_vec(int64_t n, const int32_t *ptr, const int32_t *src, const double *vals, double *out,
                       hipStream_t st);
void launch_dirichletize(int64_t n, const int32_t *rowptr, const int32_t *col, const uint8_t *dir, double *val,
                         int diag_one, hipStream_t st);
void launch_lift_finish(int64_t n, const uint8_t *dir, double *y, hipStream_t st);
void launch_expand_dirichlet(int64_t n, const uint8_t *dir, const double *gvals, double *x, hipStream_t st);
void launch_diag_extract(int64_t n, const int32_t *rowptr, const int32_t *col, const double *val, double *d,
                         hipStream_t st);
void launch_target_rhs(int dim, int p, int64_t ncells, int n_loc, const LocalFn *fns, const int32_t *cell_dofs,
                       const double *h, const double *lo, const int32_t *ncell3, const double *tlo,
                       const double *thi, const double *E, const uint8_t *dir, double *rhs_cells,
                       double *Jcells, hipStream_t st);
void launch_cell_gradient(int dim, int64_t ncells, int n_loc, const FeTables &T, const int32_t *cell_dofs,
                          const double *h, const double *mu, const double *E, const double *lam, double *grad,
                          hipStream_t st);
void launch_sum(const double *x, int64_t n, double *out, hipStream_t st);

// ---- domain decomposition and small helpers (kernels_ddm.hip)
void launch_ddm_rhs(int64_t ntouch, const int32_t *touch_sys, const int32_t *touch_dof, const int32_t *touch_ptr,
                    const int32_t *touch_src, double *const *rhs, const double *G, hipStream_t st);
// G update of eq. (8) with S = s 1 (s = s_re + i s_im): u_e = -G[rev(e)] - 2 i k w s (M_Sigma E)[e]
void launch_ddm_update(int64_t nent, const int32_t *ent_sys, const int32_t *ent_row, const int32_t *ent_rev,
                       const int32_t *ent_mptr, const int32_t *m_col, const double *m_val,
                       const double *const *X, const double *G, double kw, double s_re, double s_im, int mode,
                       double *out, hipStream_t st);
void launch_ddm_glue(int64_t n, const int32_t *own_sys, const int32_t *own_loc, const double *const *X, double *E,
                     hipStream_t st);
void launch_diag_solve(int64_t n, const double *d, const double *r, double *z, hipStream_t st);
void launch_dot1(int64_t m, const double *a, const double *b, double *out, hipStream_t st);
void launch_cg_step(int64_t m, int mode, const double *sc, double *x, const double *p, double *r, const double *q,
                    double *pp, const double *z, hipStream_t st);

}  // namespace thm
