// Internal solver structures: the assembled system, the batched GMRES workspace and
// the per-call batched solve context.
#pragma once
#include <functional>
#include <map>
#include <memory>

#include "kernels.h"

namespace thm {
struct Ddm;

// Exact factorised K^{-1} (condensation + block cyclic reduction), shareable by
// systems with identical matrices.
struct Factor {
    int nlayers = 0;
    bool lu = false;             // block-LU form (thick layers) instead of cyclic reduction
    std::vector<int32_t> bsize;
    std::vector<int64_t> boff;
    int n_int = 0, ne = 0;
    int64_t n_cells = 0;
    std::vector<int64_t> pboff;  // padded layer offsets of the skeleton work vectors
    int64_t sp = 0;              // padded skeleton length (positions per member column)
    DBuf<double> kiinv, F, FT;     // kiinv stored transposed per cell after setup (see PrecDesc)
    DBuf<float> kiinv32, F32, FT32;
    DBuf<double> mat;            // apply matrices during setup (rows x cols, segments packed)
    DBuf<double> matp;           // apply matrices, padded (rows x ld, segments aligned)
    DBuf<float> matp32;
    struct Blk {
        int layer;
        int64_t off;             // in mat
        int64_t poff;            // in matp / matp32
        int rows, cols, nseg;
        int ld;                  // padded row length (multiple of BCR_KS)
        int seg_layer[SEGMAX], seg_src[SEGMAX];
        int seg_pstart[SEGMAX + 1];  // padded column of each segment; [nseg] = padded width
        int out_dst, subtract;
    };
    std::vector<std::vector<Blk>> fwd, bwd;   // per level
    std::vector<std::map<int, int>> fw_at, bk_at;
    std::vector<std::vector<int>> level_pos;
    // The reduction stops when few blocks remain; their block-tridiagonal system is
    // inverted densely and applied as one phase (one task per block row).  The block-LU
    // form has one task per forward and backward level and no dense last system.
    std::vector<Blk> tops;
    std::vector<int> top_pos;
    int64_t top_off = 0;
    int top_n = 0;
    int64_t mat_elems = 0, matp_elems = 0, bytes = 0;
    double setup_ms = 0.0;
};
}

// One assembled problem (global or one subdomain).  Owns all device memory.
struct thm_system {
    thm_problem prob{};
    std::vector<double> mu_host;
    std::vector<double> eps_host;  // empty: eps = 1
    uint32_t iface_sides = 0;  // sides that are DDM interfaces (impedance with k w)
    thm::Topo topo;
    thm::HostCSR K, C, Minc;
    std::vector<thm::Side> sides_c, sides_inc;  // sides carrying C; Gamma^inc sides
    std::vector<uint8_t> dir;
    thm::Layering L;
    int64_t n = 0, n_free = 0;
    int nf = 0;  // local functions per side

    thm::DBuf<thm::LocalFn> fns;
    thm::FeTables tcell, tside, tload;
    thm::DBuf<int32_t> cell_dofs, k_rowptr, k_col, k_gptr, k_gsrc, c_rowptr, c_col, c_gptr, c_gsrc;
    thm::DBuf<int32_t> side_fn, sc_axis, sc_side, sc_cell, si_axis, si_side, si_cell;
    thm::DBuf<double> h, lo;
    thm::DBuf<int32_t> ncell;
    thm::DBuf<double> mu_d, eps_d;
    thm::DBuf<double> kel, kraw, kval, craw, cval;
    // tangential trace mass blocks of the sides carrying C (sides_c order, nf x nf each) and the
    // range of sides_c of each (axis, side) group (DDM interface sides with S = s 1 add to K)
    thm::DBuf<double> cside;
    int cside_lo[6] = {0, 0, 0, 0, 0, 0}, cside_hi[6] = {0, 0, 0, 0, 0, 0};
    thm::DBuf<float> kval32, cval32;
    thm::DBuf<int32_t> sl_ptr, sl_col, sl_src, sl_row;  // K in SELL-64 (see MatDesc)
    thm::DBuf<double> sl_val;
    thm::DBuf<float> sl_val32;
    thm::DBuf<uint8_t> dir_d;
    thm::DBuf<double> gD, rhs;  // complex, full length (2n doubles)
    thm::DBuf<int32_t> d2c_ptr, d2c_src;

    // preconditioner: skeleton maps of this system and the (possibly shared) factor
    thm::DBuf<int32_t> Lskel_dof, Lskel_pos, Ldof_pos, Lcell_pos, Lcond_ptr, Lcond_cell, Lcond_loc;
    std::shared_ptr<thm::Factor> fac;

    // domain decomposition
    std::vector<std::unique_ptr<thm_system>> subs;
    std::unique_ptr<thm::Ddm> ddm;

    ~thm_system();
};

namespace thm {

struct Krylov {
    Batch B;
    int m = 50;
    DBuf<double> H, cs, sn, g, y, hcol, hcol2, hnext, bnorm, beta, resid, est, part;
    DBuf<double> rtol_d;  // Arnoldi stopping tolerance, read by the (captured) finish kernel
    double rtol_h = 0.0;  // host copy (source of the async upload; lives with the workspace)
    DBuf<int32_t> running, active, jcnt, iters;
    DBuf<double> V64, w64, z64, cur64;
    DBuf<float> V32, w32, z32, cur32;
    // preconditioned basis Z = P^{-1} V (m columns), kept when the preconditioner is costly
    // relative to the step count (flexible form: x += Z y at the end of a cycle)
    DBuf<double> Z64;
    DBuf<float> Z32;
    static constexpr int NEV = 8;
    // Arnoldi steps per captured graph: the host launches a cycle as chunks of this many steps
    static constexpr int GRAPH_SPC = 8;
    int32_t *pinned = nullptr;  // NEV x ns host flags (coherent host memory, written by kernels)
    int32_t *pinned_dev = nullptr;  // the same memory as seen by kernels
    int32_t *pinned_run = nullptr, *pinned_run_dev = nullptr;  // ns running flags of the current cycle
    DBuf<int32_t> step_ctr;     // Arnoldi steps of the current cycle (selects the flag slot)
    hipEvent_t ev[NEV] = {};
    struct GraphSlot {
        hipGraphExec_t exec = nullptr;
        hipGraph_t graph = nullptr;
        int key_T = -1, orth = -1, max_iter = -1, cplx = -1, pkind = -1;
        float csign = 0.f;
        double rtol = -1.0;
        const void *owner = nullptr;
        const void *b = nullptr, *x = nullptr;  // vectors baked into a cycle-turn graph
    } slots[8][2];  // [precision, sign, preconditioner kind][chunk of steps, cycle turn]
    void init(const std::vector<int64_t> &n, int m, hipStream_t st);
    template <class T> T *V();
    template <class T> T *w();
    template <class T> T *z();
    template <class T> T *cur();
    template <class T> T *Z();
    template <class T> void ensure(hipStream_t st);
    template <class T> void ensure_z();
    void drop_graphs();
    ~Krylov();
};

template <class T>
struct KOps {
    // y = A x (b == nullptr) or y = b - A x, for systems with mask set
    std::function<void(const T *x, T *y, const T *b, const int32_t *mask)> apply;
    // y = P^{-1} x
    std::function<void(const T *x, T *y, const int32_t *mask)> prec;
    // optional pair for the Arnoldi step of a batch with shared-K groups: prec_i is prec that
    // also writes the member-interleaved copy of y, and apply_i is y = A x reading x from it
    std::function<void(const T *x, T *y, const int32_t *mask)> prec_i;
    std::function<void(T *y, const int32_t *mask)> apply_i;
    bool graphable = false;
    const void *owner = nullptr;  // identity of the operator (graph cache key)
    float csign = 1.f;
    int pkind = 0;                // preconditioner: 0 block diag(K, K)^{-1}, 1 complete (K +- iC)^{-1};
                                  // 2, 3: the same two applied in FP32 inside FP64 GMRES (GMRES-IR)
};

struct GmresParams {
    double rtol = 1e-8;
    int max_iter = 5000;
    int orth = THM_ORTH_CGS;
    bool use_graph = true;
    int cplx = 1;  // complex-scalar Arnoldi (1) or real-scalar (0)
};

template <class T>
void gmres_run(Krylov &K, const KOps<T> &ops, const T *b, T *x, const int32_t *mask_in, const GmresParams &p,
               hipStream_t st);

// Batched solve context over assembled (sub)systems.
struct Ctx {
    std::vector<thm_system *> sys;
    int ns = 0;
    hipStream_t st = nullptr;
    Krylov K;
    PrecBatch P;
    DBuf<MatDesc> mat64, mat32;
    DBuf<const uint8_t *> dirs;
    DBuf<double> x64, b64, r64, ws64, ys64, tw64;
    DBuf<float> x32, b32, ws32, ys32, tw32;
    DBuf<int32_t> mask_all, run_ir, ir_aux;
    DBuf<double> ir_scal;
    int64_t fp64_fallbacks = 0;  // systems finished in FP64 after GMRES-IR missed rtol (cumulative)
    std::vector<int32_t> last_fb;  // per system, last solve: finished by FP64 GMRES with the FP64 factor
    std::vector<int32_t> last_ir;  // per system, last solve: finished by GMRES-IR (FP64 Krylov, FP32 factor)
    DBuf<float> mx32, my32;        // FP32 copies of the GMRES-IR preconditioner's input and output
    // per system: a classical refinement step failed to contract in this context, so its later
    // THM_FP32_IR solves go straight to GMRES-IR (the context is rebuilt when K changes)
    std::vector<int32_t> ir_sticky[2];  // per preconditioner kind (block, complete inverse)
    DBuf<double> rnorm, bnorm64, resid64;
    int lpr64 = 81, lpr32 = 81;  // SpMV variants (10 * lanes_per_row + unroll, or a SELL code)
    // groups of systems with the same K for the grouped SELL product (SPMV_SELL_GROUP)
    DBuf<SpmvGroup> sgroups;
    std::vector<SpmvGroup> hgroups;  // host copy (crow points to device memory)
    DBuf<uint8_t> sgcrow;
    Sched gsched;
    int ngroups = 0;
    bool spmv_shared = false;  // some group has two or more members
    int64_t xi_total = 0;      // complex entries of the member-interleaved copy (see SpmvGroup::xoff)
    Sched ilsched;             // blocks of the preconditioner's interleaved output, per group
    DBuf<double> xi64;
    DBuf<float> xi32;
    void ensure_xi(bool f32);  // allocates (and zeroes) the interleaved copy of one precision
    void build_groups();
    // y = A x or y = b - A x with SpMV variant v (a code of launch_spmv or SPMV_SELL_GROUP)
    template <class T> void spmv(int v, const int32_t *mask, const T *x, T *y, const T *b, float csign);

    bool prec_ready = false;

    // complete inverse (K + iC)^{-1} = K^{-1} - K^{-1} P^T M^{-1} (i C_G P) K^{-1} (see kernels_full.hip)
    struct Full {
        bool ready = false;
        FullDesc d;
        std::vector<int64_t> r;                     // boundary size per system
        int nunique = 0;                            // distinct M^{-1} stored
        DBuf<int64_t> goff, moff;
        DBuf<int32_t> gam, cptr, ccol;
        DBuf<double> cval64, m64, u64, part64, w64, y64, neg1;
        DBuf<float> cval32, m32, u32, part32, w32, y32;
        int64_t bytes = 0;                          // M^{-1} storage, FP64 + FP32
        double setup_ms = 0.0;
    } full;
    void build_full();

    // spmv_setup: form the SpMV groups and run the SpMV autotuner (not needed by a context
    // that only applies the preconditioner)
    void build(const std::vector<thm_system *> &s, int m, hipStream_t stream, bool spmv_setup = true);
    void build_prec();
    // operator (and, unless with_prec is false, preconditioner) of the batch; pkind selects
    // the block preconditioner (0) or the complete inverse (1)
    KOps<double> ops64(float csign, bool with_prec = true, int pkind = 0);
    KOps<float> ops32(float csign, bool with_prec = true, int pkind = 0);
    // FP64 operator with the block preconditioner applied by the FP32 factor (input rounded to
    // FP32, output widened): the correction solve of GMRES-based iterative refinement
    KOps<double> ops_mixed(float csign, int pk = 0);
    // y = P^{-1} x with the FP32 factor: block diag(K, K)^{-1} (pkind 0) or the complete
    // inverse (pkind 1, transpose sign csign < 0)
    void prec32(int pkind, float csign, const float *x, float *y, const int32_t *mask);
    // Solve A x = b for the systems in mask (device, nullable = all); b64/x64 slots hold
    // the right-hand sides and initial guesses (zero on Dirichlet rows).
    void solve(const thm_solve_opts &o, float csign, const int32_t *mask, std::vector<int> &iters,
               std::vector<int> &refines, std::vector<double> &resid);
    void autotune();
    // Time `reps` applications of the cyclic-reduction phases (k_bcr_mfma launches only)
    // with HIP events on this context's stream; returns ms per application, and the
    // algorithmic bytes and number of launches per application.
    double time_bcr(int prec, int reps, double *bytes, int *launches);
    std::vector<double> bcr_bytes[2];  // per phase, per precision (matrix once + member vectors)
    void copy_in(int s, const double *src_dev, double *slot);
    void copy_out(int s, const double *slot, double *dst_dev);
};

void setup_precond(const std::vector<thm_system *> &systems, hipStream_t st, bool share = true);
// Same mesh, degree, Dirichlet set, K pattern and (bitwise) K values and element matrices:
// the systems share a preconditioner factor and one read of K in the grouped SpMV.
bool same_matrices(thm_system &a, thm_system &b, hipStream_t st);
double now_ms();

// Allocation-free block-preconditioner apply (noalloc.hip): y = diag(K, K)^{-1} x for the
// single system of context c, on stream st, with every work vector in the library's static
// device scratch array of NOALLOC_SCRATCH_BYTES.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
void noalloc_prec_apply(Ctx &c, int precision, const double *x, double *y, hipStream_t st);

}  // namespace thm
