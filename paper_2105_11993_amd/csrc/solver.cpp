// Batched block-preconditioned GMRES on the real 2x2 block system (Sec. 3.2,
// eq. (4), eq. (11)), its FP32 + FP64-refinement form, the preconditioner setup and
// the SpMV schedule autotuner.
//
// GMRES (readings of the paper): right preconditioning, restart m, classical
// Gram-Schmidt (optionally twice), Hessenberg and Givens rotations in FP64, stop on
// the true relative residual ||b - A x|| / ||b|| checked at each restart and on the
// Givens estimate inside a cycle.  Every kernel serves all systems of a batch;
// converged systems drop out through device-side flags.  One Arnoldi step is
// captured once as a hipGraph and replayed (its kernels read the step index from
// device memory), and the host polls convergence one step behind the device.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>

#include "solver.h"

namespace thm {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ Krylov workspace
void Krylov::init(const std::vector<int64_t> &n, int m_, hipStream_t st) {
    drop_graphs();
    m = m_;
    B.init(n, 2 * (m + 1) + 2, st);
    const int ns = B.ns;
    H.alloc((size_t)ns * 2 * (m + 1) * m);  // complex, column-major (m+1) x m
    cs.alloc((size_t)ns * m);
    sn.alloc((size_t)ns * 2 * m);
    g.alloc((size_t)ns * 2 * (m + 1));
    y.alloc((size_t)ns * 2 * (m + 1));
    hcol.alloc((size_t)ns * 2 * (m + 1));
    hcol2.alloc((size_t)ns * 2 * (m + 1));
    for (DBuf<double> *b : {&hnext, &bnorm, &beta, &resid, &est}) b->alloc(ns);
    rtol_d.alloc(1);
    part.alloc((size_t)std::max(1, B.vs.nblocks) * NPW * B.maxcols);
    for (DBuf<int32_t> *b : {&running, &active, &jcnt, &iters}) b->alloc(ns);
    if (pinned) (void)hipHostFree(pinned);
    THM_HIP(hipHostMalloc((void **)&pinned, sizeof(int32_t) * (NEV + 1) * std::max(ns, 1),
                          hipHostMallocMapped | hipHostMallocCoherent));
    THM_HIP(hipHostGetDevicePointer((void **)&pinned_dev, pinned, 0));
    pinned_run = pinned + (size_t)NEV * std::max(ns, 1);
    pinned_run_dev = pinned_dev + (size_t)NEV * std::max(ns, 1);
    step_ctr.alloc(1);
    for (auto &e : ev)
        if (!e) THM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

template <> double *Krylov::V<double>() { return V64.p; }
template <> float *Krylov::V<float>() { return V32.p; }
template <> double *Krylov::w<double>() { return w64.p; }
template <> float *Krylov::w<float>() { return w32.p; }
template <> double *Krylov::z<double>() { return z64.p; }
template <> float *Krylov::z<float>() { return z32.p; }
template <> double *Krylov::cur<double>() { return cur64.p; }
template <> float *Krylov::cur<float>() { return cur32.p; }
template <> double *Krylov::Z<double>() { return Z64.p; }
template <> float *Krylov::Z<float>() { return Z32.p; }
template <> void Krylov::ensure_z<double>() {
    if (!Z64.n) Z64.alloc((size_t)m * B.Ltot);
}
template <> void Krylov::ensure_z<float>() {
    if (!Z32.n) Z32.alloc((size_t)m * B.Ltot);
}

template <>
void Krylov::ensure<double>(hipStream_t) {
    if (V64.n) return;
    V64.alloc((size_t)(m + 1) * B.Ltot);
    w64.alloc(B.Ltot);
    z64.alloc(B.Ltot);
    cur64.alloc(B.Ltot);
}
template <>
void Krylov::ensure<float>(hipStream_t) {
    if (V32.n) return;
    V32.alloc((size_t)(m + 1) * B.Ltot);
    w32.alloc(B.Ltot);
    z32.alloc(B.Ltot);
    cur32.alloc(B.Ltot);
}

void Krylov::drop_graphs() {
    for (auto &row : slots)
        for (auto &s : row) {
            if (s.exec) (void)hipGraphExecDestroy(s.exec);
            if (s.graph) (void)hipGraphDestroy(s.graph);
            s = GraphSlot{};
        }
}

Krylov::~Krylov() {
    drop_graphs();
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (pinned) (void)hipHostFree(pinned);
}

// ------------------------------------------------------------------ GMRES
template <class T> struct TypeKey;
template <> struct TypeKey<double> { static constexpr int v = 0; };
template <> struct TypeKey<float> { static constexpr int v = 1; };

// The complete inverse (pkind 1, 3) costs a step's worth of work per application and its
// solves take a step or two: GMRES keeps Z = P^{-1} V and ends a cycle with x += Z y instead of
// applying the preconditioner once more (flexible form; the same iterates for a fixed
// preconditioner).
template <class T>
static bool flexible(const KOps<T> &ops) {
    return ops.pkind == 1 || ops.pkind == 3;
}

template <class T>
static void arnoldi_step(Krylov &K, const KOps<T> &ops, const GmresParams &p, int spc, hipStream_t st) {
    Batch &B = K.B;
    const int m = K.m;
    T *V = K.V<T>(), *w = K.w<T>(), *z = K.z<T>(), *cur = K.cur<T>();
    int32_t *act = K.active.p;
    if (ops.apply_i) {
        ops.prec_i(cur, z, act);
        ops.apply_i(w, act);
    } else {
        ops.prec(cur, z, act);
        ops.apply(z, w, nullptr, act);
    }
    if (flexible(ops)) launch_scale<T, T>(B, act, nullptr, 0, z, K.Z<T>(), K.jcnt.p, B.Ltot, nullptr, st);
    const int ldh = 2 * (m + 1);
    launch_dots<T>(B, act, K.jcnt.p, V, B.Ltot, w, K.part.p, p.cplx, st);
    launch_reduce_cols(B, act, K.jcnt.p, 0, K.part.p, K.hcol.p, ldh, 0, st);
    launch_cgs_update<T>(B, act, K.jcnt.p, V, B.Ltot, w, K.hcol.p, ldh, K.part.p, st);
    if (p.orth == THM_ORTH_CGS2) {
        launch_dots<T>(B, act, K.jcnt.p, V, B.Ltot, w, K.part.p, p.cplx, st);
        launch_reduce_cols(B, act, K.jcnt.p, 0, K.part.p, K.hcol2.p, ldh, 0, st);
        launch_reduce_cols(B, act, K.jcnt.p, 0, K.part.p, K.hcol.p, ldh, 1, st);
        launch_cgs_update<T>(B, act, K.jcnt.p, V, B.Ltot, w, K.hcol2.p, ldh, K.part.p, st);
    }
    launch_arnoldi_finish(B, K.part.p, act, K.jcnt.p, K.hcol.p, ldh, K.H.p, K.cs.p, K.sn.p, K.g.p, K.hnext.p,
                          K.bnorm.p, K.rtol_d.p, m, K.iters.p, p.max_iter, K.est.p, K.pinned_dev, K.step_ctr.p, spc,
                          Krylov::NEV, st);
    launch_scale<T, T>(B, act, K.hnext.p, 1, w, V, K.jcnt.p, B.Ltot, cur, st, K.step_ctr.p);
}

// Start of a cycle: w = b - A x, beta = ||w||, stop test (running flags to host memory),
// V_0 = cur = w / beta, step counter reset.
template <class T>
static void cycle_open(Krylov &K, const KOps<T> &ops, const GmresParams &p, const T *b, const T *x,
                       hipStream_t st) {
    Batch &B = K.B;
    T *V = K.V<T>(), *w = K.w<T>(), *cur = K.cur<T>();
    ops.apply(x, w, b, K.running.p);
    launch_norm2<T>(B, K.running.p, w, K.part.p, st);
    launch_cycle_start(B, K.part.p, K.running.p, K.active.p, K.jcnt.p, K.bnorm.p, K.rtol_d.p, K.g.p, K.m,
                       K.beta.p, K.resid.p, K.iters.p, p.max_iter, K.step_ctr.p, K.pinned_run_dev, st);
    launch_scale<T, T>(B, K.active.p, K.beta.p, 1, w, V, K.jcnt.p, B.Ltot, cur, st);
}

// End of a cycle: y = H^{-1} g, x += P^{-1} (V y).
template <class T>
static void cycle_close(Krylov &K, const KOps<T> &ops, T *x, hipStream_t st) {
    Batch &B = K.B;
    T *V = K.V<T>(), *z = K.z<T>(), *cur = K.cur<T>();
    launch_hsolve(B, K.running.p, K.jcnt.p, K.H.p, K.g.p, K.y.p, K.m, st);
    if (flexible(ops)) {
        launch_lincomb<T>(B, K.running.p, K.jcnt.p, K.Z<T>(), B.Ltot, K.y.p, 2 * (K.m + 1), cur, st);
        launch_axpy<T, T>(B, K.running.p, nullptr, cur, x, st);
        return;
    }
    launch_lincomb<T>(B, K.running.p, K.jcnt.p, V, B.Ltot, K.y.p, 2 * (K.m + 1), cur, st);
    ops.prec(cur, z, K.running.p);
    launch_axpy<T, T>(B, K.running.p, nullptr, z, x, st);
}

// Arnoldi steps per chunk graph: GRAPH_SPC, or one step where a solve takes only a step or
// two (the complete inverse), so that few steps run past convergence.
template <class T>
static int chunk_steps(const KOps<T> &ops) {
    return flexible(ops) ? 1 : Krylov::GRAPH_SPC;
}

// Captured once per (precision, operator, options, kind, vectors) and replayed: kind 0 is a
// chunk of chunk_steps() Arnoldi steps, kind 1 closes a cycle and opens the next (b and x are
// part of the key, their addresses being baked into the graph).
template <class T>
static hipGraphExec_t cycle_graph(Krylov &K, const KOps<T> &ops, const GmresParams &p, int kind, const T *b, T *x,
                                  hipStream_t st) {
    const int key = TypeKey<T>::v * 2 + (ops.csign < 0 ? 1 : 0) + (ops.pkind >= 2 ? 4 : 0);
    Krylov::GraphSlot &s = K.slots[key][kind];
    if (s.exec && s.owner == ops.owner && s.orth == p.orth && s.max_iter == p.max_iter && s.cplx == p.cplx &&
        s.pkind == ops.pkind && (kind == 0 || (s.b == (const void *)b && s.x == (const void *)x)))
        return s.exec;
    const int spc = chunk_steps(ops);
    if (s.exec) (void)hipGraphExecDestroy(s.exec);
    if (s.graph) (void)hipGraphDestroy(s.graph);
    s = Krylov::GraphSlot{};
    THM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
        if (kind == 0) {
            for (int i = 0; i < spc; ++i) arnoldi_step<T>(K, ops, p, spc, st);
        } else {
            cycle_close<T>(K, ops, x, st);
            cycle_open<T>(K, ops, p, b, x, st);
        }
    } catch (...) {
        hipGraph_t g;
        (void)hipStreamEndCapture(st, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    THM_HIP(hipStreamEndCapture(st, &s.graph));
    THM_HIP(hipGraphInstantiate(&s.exec, s.graph, nullptr, nullptr, 0));
    s.owner = ops.owner;
    s.orth = p.orth;
    s.rtol = p.rtol;
    s.max_iter = p.max_iter;
    s.cplx = p.cplx;
    s.pkind = ops.pkind;
    s.csign = ops.csign;
    s.key_T = TypeKey<T>::v;
    s.b = b;
    s.x = x;
    return s.exec;
}

static bool any_set(const volatile int32_t *h, int ns) {
    for (int i = 0; i < ns; ++i)
        if (h[i]) return true;
    return false;
}

template <class T>
void gmres_run(Krylov &K, const KOps<T> &ops, const T *b, T *x, const int32_t *mask_in, const GmresParams &p,
               hipStream_t st) {
    Batch &B = K.B;
    const int ns = B.ns, m = K.m;
    K.ensure<T>(st);
    if (flexible(ops)) K.ensure_z<T>();
    launch_norm2<T>(B, mask_in, b, K.part.p, st);
    launch_norm_finish(B, K.part.p, mask_in, K.bnorm.p, nullptr, 0.0, nullptr, nullptr, st);
    THM_HIP(hipMemcpyAsync(K.running.p, mask_in, sizeof(int32_t) * ns, hipMemcpyDeviceToDevice, st));
    THM_HIP(hipMemsetAsync(K.iters.p, 0, sizeof(int32_t) * ns, st));
    K.rtol_h = p.rtol;
    THM_HIP(hipMemcpyAsync(K.rtol_d.p, &K.rtol_h, sizeof(double), hipMemcpyHostToDevice, st));
    const bool graph = p.use_graph && ops.graphable;
    if (!graph) {
        // host-driven: one launch sequence per Arnoldi step; the finish kernel of step j writes
        // the systems' flags to host slot j mod NEV, and the host checks the flags of step
        // j - LAG while later steps run
        for (;;) {
            cycle_open<T>(K, ops, p, b, x, st);
            THM_HIP(hipStreamSynchronize(st));
            if (!any_set(K.pinned_run, ns)) break;
            constexpr int LAG = 3;
            static_assert(LAG + 1 < Krylov::NEV, "flag slots in flight must not wrap");
            for (int step = 0; step < m; ++step) {
                arnoldi_step<T>(K, ops, p, 1, st);
                const int sl = step % Krylov::NEV;
                THM_HIP(hipEventRecord(K.ev[sl], st));
                if (step >= LAG) {
                    const int ol = (step - LAG) % Krylov::NEV;
                    THM_HIP(hipEventSynchronize(K.ev[ol]));
                    if (!any_set(K.pinned + (size_t)ol * ns, ns)) break;
                }
            }
            cycle_close<T>(K, ops, x, st);
        }
        return;
    }
    // graph replay: a cycle is ceil(m / spc) chunk graphs (steps past a system's end of cycle
    // find it inactive and do nothing) and one close-and-reopen graph.  The finish kernels of
    // chunk c leave the systems' flags in host slot c mod NEV; the host checks chunk c - 1
    // while chunk c runs, and the running flags once per cycle.
    hipGraphExec_t chunk = cycle_graph<T>(K, ops, p, 0, b, x, st);
    hipGraphExec_t turn = cycle_graph<T>(K, ops, p, 1, b, x, st);
    cycle_open<T>(K, ops, p, b, x, st);
    THM_HIP(hipStreamSynchronize(st));
    const int spc = chunk_steps(ops);
    const int nchunks = (m + spc - 1) / spc;
    static_assert(Krylov::NEV >= 4, "chunk flag slots in flight must not wrap");
    while (any_set(K.pinned_run, ns)) {
        for (int c = 0; c < nchunks; ++c) {
            THM_HIP(hipGraphLaunch(chunk, st));
            THM_HIP(hipEventRecord(K.ev[c % Krylov::NEV], st));
            if (c >= 1) {
                const int ol = (c - 1) % Krylov::NEV;
                THM_HIP(hipEventSynchronize(K.ev[ol]));
                if (!any_set(K.pinned + (size_t)ol * ns, ns)) break;
            }
        }
        THM_HIP(hipGraphLaunch(turn, st));
        THM_HIP(hipStreamSynchronize(st));
    }
}

template void gmres_run<double>(Krylov &, const KOps<double> &, const double *, double *, const int32_t *,
                                const GmresParams &, hipStream_t);
template void gmres_run<float>(Krylov &, const KOps<float> &, const float *, float *, const int32_t *,
                               const GmresParams &, hipStream_t);

void bcr_chunk_table(const BcrTask &t, std::vector<int32_t> &out) {
    const int nch = t.ld / 8, nvalid = t.seg_pstart[t.nseg] / 8;
    out.assign(nch, 0);
    int q = 0;
    for (int kc = 0; kc < nch; ++kc) {
        const int kk = std::min(kc, nvalid - 1);
        while (q + 1 < t.nseg && 8 * kk >= t.seg_pstart[q + 1]) ++q;
        // column 8 kc reads position seg_off + (8 kk - pstart) = delta + 8 kc
        const int64_t delta = t.seg_off[q] - t.seg_pstart[q] + 8 * (int64_t)(kk - kc);
        if (2 * delta > INT32_MAX || 2 * delta < INT32_MIN)
            fail(THM_EUNSUPPORTED, "skeleton work vector too long for the apply kernel");
        out[kc] = (int32_t)(2 * delta) | (t.seg_src[q] & 1);
    }
}

// ------------------------------------------------------------------ batched context
void Ctx::build(const std::vector<thm_system *> &s, int m, hipStream_t stream, bool spmv_setup) {
    sys = s;
    ns = (int)s.size();
    st = stream;
    std::vector<int64_t> n(ns);
    for (int i = 0; i < ns; ++i) n[i] = sys[i]->n;
    K.init(n, m, st);
    std::vector<MatDesc> h64(ns), h32(ns);
    std::vector<const uint8_t *> hd(ns);
    for (int i = 0; i < ns; ++i) {
        const thm_system &S = *sys[i];
        h64[i] = {S.n, S.k_rowptr.p, S.k_col.p, S.kval.p, S.c_rowptr.p, S.c_col.p, S.cval.p,
                  S.sl_ptr.p, S.sl_col.p, S.sl_row.p, S.sl_val.p};
        h32[i] = {S.n, S.k_rowptr.p, S.k_col.p, S.kval32.p, S.c_rowptr.p, S.c_col.p, S.cval32.p,
                  S.sl_ptr.p, S.sl_col.p, S.sl_row.p, S.sl_val32.p};
        hd[i] = S.dir_d.p;
    }
    mat64.upload(h64, st);
    mat32.upload(h32, st);
    dirs.upload(hd, st);
    x64.alloc(K.B.Ltot);
    b64.alloc(K.B.Ltot);
    r64.alloc(K.B.Ltot);
    THM_HIP(hipMemsetAsync(x64.p, 0, sizeof(double) * x64.n, st));
    THM_HIP(hipMemsetAsync(b64.p, 0, sizeof(double) * b64.n, st));
    THM_HIP(hipMemsetAsync(r64.p, 0, sizeof(double) * r64.n, st));
    mask_all.upload(std::vector<int32_t>(ns, 1), st);
    run_ir.alloc(ns);
    rnorm.alloc(ns);
    bnorm64.alloc(ns);
    resid64.alloc(ns);
    THM_HIP(hipStreamSynchronize(st));
    if (!spmv_setup) return;
    build_groups();
    autotune();
}

// Groups of systems with the same K, in batch order, at most SPMV_GMAX each.
void Ctx::build_groups() {
    std::vector<std::vector<int>> mem;
    std::vector<int> rep;
    for (int i = 0; i < ns; ++i) {
        int g = -1;
        for (size_t q = 0; q < rep.size() && g < 0; ++q)
            if ((int)mem[q].size() < SPMV_GMAX && same_matrices(*sys[rep[q]], *sys[i], st)) g = (int)q;
        if (g < 0) {
            rep.push_back(i);
            mem.emplace_back();
            g = (int)rep.size() - 1;
        }
        mem[g].push_back(i);
    }
    ngroups = (int)rep.size();
    spmv_shared = false;
    std::vector<int64_t> coff(ngroups + 1, 0), rows(ngroups), waves(ngroups), xoff(ngroups + 1, 0);
    for (int g = 0; g < ngroups; ++g) {
        rows[g] = sys[rep[g]]->n;
        waves[g] = (rows[g] + SELL_C - 1) / SELL_C * (int64_t)(((int)mem[g].size() + 3) / 4);
        coff[g + 1] = coff[g] + ((rows[g] + 255) & ~int64_t(255));
        spmv_shared |= mem[g].size() > 1;
        // interleaved copy: rows x npad complex entries per group, groups 16-entry aligned
        xoff[g + 1] = (xoff[g] + rows[g] * (((int64_t)mem[g].size() + 3) & ~int64_t(3)) + 15) & ~int64_t(15);
    }
    xi_total = xoff[ngroups];
    {
        // interleaved preconditioner output: blocks of IL_TILE DoFs of every member of a group
        std::vector<int64_t> nb(ngroups);
        for (int g = 0; g < ngroups; ++g) nb[g] = (rows[g] + IL_TILE - 1) / IL_TILE;
        ilsched.build(nb, 1, st);
    }
    std::vector<uint8_t> crow(coff[ngroups], 0);
    for (int g = 0; g < ngroups; ++g)
        for (int i : mem[g]) {
            const std::vector<int32_t> &rp = sys[i]->C.rowptr;
            for (int64_t r = 0; r < rows[g]; ++r)
                if (rp[r + 1] > rp[r]) crow[coff[g] + r] = 1;
        }
    sgcrow.upload(crow, st);
    std::vector<SpmvGroup> h(ngroups);
    for (int g = 0; g < ngroups; ++g) {
        SpmvGroup &G = h[g];
        G.rep = rep[g];
        G.nm = (int32_t)mem[g].size();
        G.npad = (G.nm + 3) & ~3;
        for (int j = 0; j < SPMV_GMAX; ++j) G.mem[j] = mem[g][std::min(j, G.nm - 1)];
        G.crow = sgcrow.p + coff[g];
        G.xoff = xoff[g];
    }
    sgroups.upload(h, st);
    hgroups = h;
    gsched.build(waves, 4, st);
    THM_HIP(hipStreamSynchronize(st));
}

template <class T>
void Ctx::spmv(int v, const int32_t *mask, const T *x, T *y, const T *b, float csign) {
    const MatDesc *m = sizeof(T) == 8 ? mat64.p : mat32.p;
    if (v == SPMV_SELL_GROUP || v == SPMV_SELL_GROUP_IL) {  // outside an Arnoldi step: per-system x
        launch_spmv_group<T>(m, K.B.off.p, sgroups.p, gsched, ngroups, mask, x, y, b, csign, st);
        return;
    }
    launch_spmv<T>(v, m, K.B.off.p, K.B.spmv_sched(v, st), ns, mask, x, y, b, csign, st);
}
template void Ctx::spmv<double>(int, const int32_t *, const double *, double *, const double *, float);
template void Ctx::spmv<float>(int, const int32_t *, const float *, float *, const float *, float);

// Preconditioner of the batch: factorisation (shared between identical systems) and the
// batched apply schedule.  Built on first use, so SpMV-only uses of a context skip it.
void Ctx::build_prec() {
    if (prec_ready) return;
    setup_precond(sys, st);
    std::vector<int64_t> n(ns), nsk(ns);
    for (int i = 0; i < ns; ++i) {
        n[i] = sys[i]->n;
        nsk[i] = sys[i]->L.n_skel;
    }
    std::vector<PrecDesc> p64(ns), p32(ns);
    std::vector<int64_t> soff(ns);
    // factor groups in order of first appearance
    std::vector<Factor *> groups;
    std::vector<std::vector<int32_t>> members;
    for (int i = 0; i < ns; ++i) {
        thm_system &S = *sys[i];
        Factor &f = *S.fac;
        auto it = std::find(groups.begin(), groups.end(), &f);
        if (it == groups.end()) {
            groups.push_back(&f);
            members.push_back({i});
        } else {
            members[it - groups.begin()].push_back(i);
        }
        const Topo &t = S.topo;
        PrecDesc d{};
        d.n = S.n;
        d.n_skel = S.L.n_skel;
        d.cell_off = t.cell_off;
        d.n_cells = (int32_t)t.n_cells;
        d.n_loc = t.n_loc;
        d.n_int = t.n_int;
        d.ne = t.n_loc - t.n_int;
        d.nlayers = S.L.nlayers;
        d.sp = S.L.n_skel_pad;
        d.cell_dofs = S.cell_dofs.p;
        d.skel_dof = S.Lskel_dof.p;
        d.skel_pos = S.Lskel_pos.p;
        d.cell_pos = S.Lcell_pos.p;
        d.dof_pos = S.Ldof_pos.p;
        d.cond_ptr = S.Lcond_ptr.p;
        d.cond_cell = S.Lcond_cell.p;
        d.cond_loc = S.Lcond_loc.p;

        p32[i] = d;
        d.kiinv = f.kiinv.p;
        d.F = f.F.p;
        d.FT = f.FT.p;
        p64[i] = d;
        p32[i].kiinv = f.kiinv32.p;
        p32[i].F = f.F32.p;
        p32[i].FT = f.FT32.p;
    }
    // Work vectors: one region per factor group, its members' columns interleaved by
    // 8-position chunks (see wv_pos); the member count is padded to the 8 or 16 columns
    // pairs of one block's n tiles only to keep each group's 16-lane runs aligned: lanes of
    // absent members read the chunk's first member, so the padding columns are never read.
    std::vector<int64_t> gbase(groups.size()), gcs(groups.size());
    int64_t so = 0;
    for (size_t g = 0; g < groups.size(); ++g) {
        const int nm = (int)members[g].size();
        const int nnt = nm > 8 ? 2 : 1;  // the same split as the tasks below
        const int64_t nmp = (int64_t)((nm + 8 * nnt - 1) / (8 * nnt)) * 8 * nnt;
        const int64_t sp = groups[g]->sp;
        if (sp % 8) fail(THM_EINVAL, "skeleton length not padded to 8");
        gcs[g] = 16 * nmp;
        gbase[g] = so;
        so += sp / 8 * gcs[g];
        so = (so + 63) & ~int64_t(63);
        for (int j = 0; j < nm; ++j) {
            const int i = members[g][j];
            if (p64[i].sp != sp) fail(THM_EINVAL, "members of a factor group differ in skeleton length");
            soff[i] = gbase[g] + 16 * (int64_t)j;
            p64[i].cs = p32[i].cs = gcs[g];
        }
    }
    P.ns = ns;
    P.d64.upload(p64, st);
    P.d32.upload(p32, st);
    P.soff.upload(soff, st);
    P.Stot = std::max<int64_t>(so, 64);
    P.skel.build(nsk, 256, st);
    P.dofs.build(n, 256, st);
    {
        std::vector<int64_t> units(ns), toff(ns);
        int64_t to = 0;
        for (int i = 0; i < ns; ++i) {
            const Topo &t = sys[i]->topo;
            units[i] = t.n_int > 0 ? (int64_t)t.n_cells * (t.n_loc - t.n_int) : 0;
            toff[i] = to;
            to += units[i];
        }
        P.cfr.build(units, 256, st);
        P.toff.upload(toff, st);
        P.Ttot = std::max<int64_t>(to, 1);
    }
    std::vector<int32_t> mp_host(1, 0);
    {
        std::vector<int32_t> &mp = mp_host, mm;
        for (auto &v : members) {
            mm.insert(mm.end(), v.begin(), v.end());
            mp.push_back((int32_t)mm.size());
        }
        P.memb_ptr.upload(mp, st);
        P.memb.upload(mm, st);
    }
    // cyclic-reduction phases: forward levels, last blocks, backward levels
    int nlev = 0;
    for (Factor *f : groups) nlev = std::max(nlev, (int)f->fwd.size());
    auto task = [&](const Factor &f, const Factor::Blk &b, int g, int prec) {
        BcrTask t{};
        t.M = prec ? (const void *)(f.matp32.p + b.poff) : (const void *)(f.matp.p + b.poff);
        t.rows = b.rows;
        t.ld = b.ld;
        t.nseg = b.nseg;
        t.group = g;
        t.mbeg = mp_host[g];
        t.mend = mp_host[g + 1];
        t.kq = ((b.ld + BCR_WPB - 1) / BCR_WPB + BCR_KS - 1) / BCR_KS * BCR_KS;
        const int nm = (int)members[g].size();
        t.nnt = nm > 8 ? 2 : 1;
        t.nmc = (nm + 8 * t.nnt - 1) / (8 * t.nnt);
        for (int q = 0; q <= SEGMAX; ++q) t.seg_pstart[q] = q <= b.nseg ? b.seg_pstart[q] : b.seg_pstart[b.nseg];
        for (int q = 0; q < SEGMAX; ++q) {
            t.seg_src[q] = q < b.nseg ? b.seg_src[q] : 0;
            t.seg_off[q] = q < b.nseg ? f.pboff[b.seg_layer[q]] : 0;
        }
        t.out_off = f.pboff[b.layer];
        t.out_dst = b.out_dst;
        t.subtract = b.subtract;
        t.gbase = gbase[g];
        t.cs = gcs[g];
        if (t.out_off % 8 || t.out_off + b.rows > f.sp) fail(THM_EINVAL, "apply output outside the work vectors");
        return t;
    };
    P.phases.clear();
    bcr_bytes[0].clear();
    bcr_bytes[1].clear();
    // Algorithmic bytes of a phase: every matrix element once (true, unpadded size), the
    // input segments of each member once, the output block written (and read when the
    // task subtracts).
    auto add_phase = [&](auto pick) {
        std::vector<BcrTask> t64, t32;
        std::vector<int64_t> u64, u32;
        double elems = 0.0, vec = 0.0;
        for (size_t g = 0; g < groups.size(); ++g)
            for (const Factor::Blk *b : pick(*groups[g])) {
                t64.push_back(task(*groups[g], *b, (int)g, 0));
                t32.push_back(task(*groups[g], *b, (int)g, 1));
                const int64_t rb = (b->rows + BCR_RT - 1) / BCR_RT;
                u64.push_back(rb * t64.back().nmc);
                u32.push_back(rb * t32.back().nmc);
                const double nm = (double)members[g].size();
                elems += (double)b->rows * b->cols;
                vec += nm * 2.0 * (b->cols + b->rows * (b->subtract ? 2.0 : 1.0));
            }
        if (t64.empty()) return;
        bcr_bytes[0].push_back(8.0 * (elems + vec));
        bcr_bytes[1].push_back(4.0 * (elems + vec));
        P.phases.emplace_back();
        PrecPhase &ph = P.phases.back();
        ph.ntasks = (int)t64.size();
        {
            // chunk tables (the same for both precisions)
            std::vector<int32_t> all, one;
            std::vector<int64_t> at;
            for (const BcrTask &t : t64) {
                ph.max_ld = std::max(ph.max_ld, t.ld);
                at.push_back((int64_t)all.size());
                bcr_chunk_table(t, one);
                // every chunk the kernel reads lies inside the group's positions
                const int64_t sp = groups[t.group]->sp;
                for (size_t kc = 0; kc < one.size(); ++kc) {
                    const int64_t p0 = (int64_t)(one[kc] >> 1) + 8 * (int64_t)kc;
                    if (p0 < 0 || p0 % 8 || p0 + 8 > sp) fail(THM_EINVAL, "apply input outside the work vectors");
                }
                all.insert(all.end(), one.begin(), one.end());
            }
            ph.tab.upload(all, st);
            for (size_t i = 0; i < t64.size(); ++i) t64[i].tab = t32[i].tab = ph.tab.p + at[i];
        }
        ph.tasks[0].upload(t64, st);
        ph.tasks[1].upload(t32, st);
        ph.sched[0].build(u64, 1, st);
        ph.sched[1].build(u32, 1, st);
        if (std::getenv("THM_PROGRESS")) {
            int64_t rows = 0, nb = 0;
            for (size_t i = 0; i < t32.size(); ++i) rows += t32[i].rows, nb += u32[i];
            std::fprintf(stderr, "[thm]   apply phase %zu: %d tasks, %lld rows, widest %d columns, %lld blocks, %.1f MB (FP32)\n",
                         P.phases.size() - 1, ph.ntasks, (long long)rows, ph.max_ld, (long long)nb,
                         bcr_bytes[1].back() * 1e-6);
        }
    };
    for (int lev = 0; lev < nlev; ++lev)
        add_phase([&](const Factor &f) {
            std::vector<const Factor::Blk *> v;
            if (lev < (int)f.fwd.size())
                for (const auto &b : f.fwd[lev]) v.push_back(&b);
            return v;
        });
    add_phase([&](const Factor &f) {
        std::vector<const Factor::Blk *> v;
        for (const auto &b : f.tops) v.push_back(&b);
        return v;
    });
    for (int lev = nlev - 1; lev >= 0; --lev)
        add_phase([&](const Factor &f) {
            std::vector<const Factor::Blk *> v;
            if (lev < (int)f.bwd.size())
                for (const auto &b : f.bwd[lev]) v.push_back(&b);
            return v;
        });
    ws64.alloc(P.Stot);
    ys64.alloc(P.Stot);
    tw64.alloc(2 * P.Ttot);
    THM_HIP(hipMemsetAsync(ws64.p, 0, sizeof(double) * ws64.n, st));
    THM_HIP(hipMemsetAsync(ys64.p, 0, sizeof(double) * ys64.n, st));
    THM_HIP(hipStreamSynchronize(st));
    prec_ready = true;
}

// Boundary set Gamma (rows of the Dirichlet-modified C with a nonzero entry), C_G, and
// M^{-1} = (I + i C_G S_G)^{-1} with S_G = P K^{-1} P^T, once per distinct system
// (same factor, same Gamma, same C_G).
void Ctx::build_full() {
    if (full.ready) return;
    build_prec();
    const double t0 = now_ms();
    std::vector<int64_t> goff(ns + 1, 0);
    std::vector<int32_t> gam, cptr(1, 0), ccol;
    std::vector<double> cval;
    full.r.assign(ns, 0);
    for (int s = 0; s < ns; ++s) {
        thm_system &S = *sys[s];
        const int64_t nnzc = (int64_t)S.C.col.size();
        std::vector<double> hv(nnzc);
        if (nnzc) THM_HIP(hipMemcpy(hv.data(), S.cval.p, sizeof(double) * nnzc, hipMemcpyDeviceToHost));
        std::vector<int32_t> loc(S.n, -1), rows;
        for (int64_t i = 0; i < S.n; ++i) {
            if (S.dir[i]) continue;
            bool any = false;
            for (int32_t e = S.C.rowptr[i]; e < S.C.rowptr[i + 1]; ++e) any = any || hv[e] != 0.0;
            if (any) {
                loc[i] = (int32_t)rows.size();
                rows.push_back((int32_t)i);
            }
        }
        for (int32_t i : rows) {
            gam.push_back(i);
            for (int32_t e = S.C.rowptr[i]; e < S.C.rowptr[i + 1]; ++e) {
                if (hv[e] == 0.0) continue;
                const int32_t c = loc[S.C.col[e]];
                if (c < 0) fail(THM_EUNSUPPORTED, "C couples a boundary DoF to a DoF outside the boundary set");
                ccol.push_back(c);
                cval.push_back(hv[e]);
            }
            cptr.push_back((int32_t)ccol.size());
        }
        full.r[s] = (int64_t)rows.size();
        goff[s + 1] = goff[s] + full.r[s];
    }
    // representatives: the first system of each (factor, Gamma, C_G) class
    std::vector<int> rep(ns);
    auto same = [&](int a, int b) {
        if (sys[a]->fac != sys[b]->fac || full.r[a] != full.r[b]) return false;
        const int64_t ga = goff[a], gb = goff[b], r = full.r[a];
        if (!std::equal(gam.begin() + ga, gam.begin() + ga + r, gam.begin() + gb)) return false;
        if (cptr[ga + r] - cptr[ga] != cptr[gb + r] - cptr[gb]) return false;
        for (int64_t i = 0; i <= r; ++i)
            if (cptr[ga + i] - cptr[ga] != cptr[gb + i] - cptr[gb]) return false;
        const int32_t ea = cptr[ga], eb = cptr[gb], ne = cptr[ga + r] - ea;
        return std::equal(ccol.begin() + ea, ccol.begin() + ea + ne, ccol.begin() + eb) &&
               std::equal(cval.begin() + ea, cval.begin() + ea + ne, cval.begin() + eb);
    };
    std::vector<int64_t> moff(ns, 0), soff(ns, 0);
    std::vector<int32_t> isrep(ns, 0);
    int64_t mtot = 0, maxr = 0, maxr_rep = 0;
    full.nunique = 0;
    for (int s = 0; s < ns; ++s) {
        rep[s] = s;
        for (int t = 0; t < s; ++t)
            if (rep[t] == t && same(s, t)) {
                rep[s] = t;
                break;
            }
        maxr = std::max(maxr, full.r[s]);
        if (rep[s] == s) {
            moff[s] = mtot;
            soff[s] = mtot;  // S_G (real) uses the same element offsets in its own buffer
            mtot += full.r[s] * full.r[s];
            isrep[s] = full.r[s] > 0;
            maxr_rep = std::max(maxr_rep, full.r[s]);
            ++full.nunique;
        } else {
            moff[s] = moff[rep[s]];
        }
    }
    // M is inverted densely in its real 2r x 2r form: bounded so that one inversion's three
    // buffers stay within 3 x 8 GiB and its 16 r^3 flops within a minute
    if (maxr_rep > 16384)
        fail(THM_EUNSUPPORTED, "boundary set too large for the complete inverse (more than 16384 DoFs carry C)");
    std::vector<float> cval32(cval.begin(), cval.end());
    full.goff.upload(goff, st);
    full.gam.upload(gam.empty() ? std::vector<int32_t>{0} : gam, st);
    full.cptr.upload(cptr, st);
    full.ccol.upload(ccol.empty() ? std::vector<int32_t>{0} : ccol, st);
    full.cval64.upload(cval.empty() ? std::vector<double>{0.0} : cval, st);
    full.cval32.upload(cval32.empty() ? std::vector<float>{0.f} : cval32, st);
    full.moff.upload(moff, st);
    full.m64.alloc(std::max<int64_t>(2 * mtot, 1));
    full.m32.alloc(std::max<int64_t>(2 * mtot, 1));
    FullDesc &d = full.d;
    d.maxr = (int)maxr;
    d.nchmax = (int)((maxr + 63) / 64);
    d.goff = full.goff.p;
    d.gam = full.gam.p;
    d.cptr = full.cptr.p;
    d.ccol = full.ccol.p;
    d.cval64 = full.cval64.p;
    d.cval32 = full.cval32.p;
    d.moff = full.moff.p;
    d.m64 = full.m64.p;
    d.m32 = full.m32.p;
    if (maxr_rep > 0) {
        // S_G: K^{-1} applied to unit vectors on Gamma, columns 2k and 2k + 1 from the real and
        // imaginary parts of one right-hand side.  A temporary batch holds Q copies of each
        // representative of a chunk; the copies share its factor and form one member group of the
        // apply, so one FP64 application yields 2Q columns of every representative of the chunk
        // while each factor matrix is read once per 16 copies.  Chunks bound the temporary
        // batch to TMP_DOFS complex DoFs (its vectors, not the factors, which are shared).
        DBuf<double> Sg(std::max<int64_t>(mtot, 1));
        constexpr int64_t TMP_DOFS = int64_t(8) << 20;
        std::vector<int> all_reps;
        for (int s = 0; s < ns; ++s)
            if (isrep[s]) all_reps.push_back(s);
        for (size_t c0 = 0; c0 < all_reps.size();) {
            int64_t rmax = 0, dofs = 0;
            size_t c1 = c0;
            while (c1 < all_reps.size()) {
                const int s = all_reps[c1];
                const int64_t q = std::min<int64_t>(16, (std::max(rmax, full.r[s]) + 1) / 2);
                if (c1 > c0 && (dofs + sys[s]->n) * q > TMP_DOFS) break;
                rmax = std::max(rmax, full.r[s]);
                dofs += sys[s]->n;
                ++c1;
            }
            const int Q = (int)std::min<int64_t>(16, (rmax + 1) / 2);
            std::vector<thm_system *> tsys;
            std::vector<int64_t> tgoff(1, 0), tsoff;
            std::vector<int32_t> tgam, tk;
            for (size_t c = c0; c < c1; ++c) {
                const int s = all_reps[c];
                for (int q = 0; q < Q; ++q) {
                    tsys.push_back(sys[s]);
                    tgam.insert(tgam.end(), gam.begin() + goff[s], gam.begin() + goff[s + 1]);
                    tgoff.push_back((int64_t)tgam.size());
                    tsoff.push_back(soff[s]);
                    tk.push_back(q);
                }
            }
            Ctx T;
            T.build(tsys, 1, st, false);
            T.build_prec();
            DBuf<int64_t> dtgoff, dtsoff;
            DBuf<int32_t> dtgam, dtk;
            dtgoff.upload(tgoff, st);
            dtsoff.upload(tsoff, st);
            dtgam.upload(tgam, st);
            dtk.upload(tk, st);
            FullDesc td = d;
            td.goff = dtgoff.p;
            td.gam = dtgam.p;
            DBuf<double> xin(T.K.B.Ltot), zout(T.K.B.Ltot);
            THM_HIP(hipMemsetAsync(xin.p, 0, sizeof(double) * xin.n, st));
            const int nt = T.ns;
            for (int64_t k = 0; 2 * k < rmax; k += Q) {
                launch_full_unit(td, nt, nullptr, T.K.B.off.p, dtk.p, (int)k, 1.0, xin.p, st);
                launch_prec_apply<double>(T.P, T.P.d64.p, T.K.B.off.p, nt, nullptr, xin.p, zout.p, T.ws64.p,
                                          T.ys64.p, T.tw64.p, st);
                launch_full_gather(td, nt, nullptr, T.K.B.off.p, dtk.p, (int)k, zout.p, dtsoff.p, Sg.p, st);
                launch_full_unit(td, nt, nullptr, T.K.B.off.p, dtk.p, (int)k, 0.0, xin.p, st);
            }
            THM_HIP(hipStreamSynchronize(st));
            c0 = c1;
        }
        // M = I + i C_G S_G in real form, inverted by Gauss-Jordan, then stored complex.  The
        // representatives are inverted in batches of at most INV_BATCH_ELEMS matrix entries
        // (three buffers of that size), so large boundary sets do not need all of them at once.
        std::vector<int> reps;
        for (int s = 0; s < ns; ++s)
            if (isrep[s]) reps.push_back(s);
        constexpr int64_t INV_BATCH_ELEMS = int64_t(1) << 30;  // 8 GiB per buffer
        DBuf<int32_t> status(1);
        THM_HIP(hipMemsetAsync(status.p, 0, sizeof(int32_t), st));
        for (size_t q0 = 0; q0 < reps.size();) {
            size_t q1 = q0;
            int64_t btot = 0;
            while (q1 < reps.size()) {
                const int64_t e = 4 * full.r[reps[q1]] * full.r[reps[q1]];
                if (q1 > q0 && btot + e > INV_BATCH_ELEMS) break;
                btot += e;
                ++q1;
            }
            DBuf<double> Bm(btot), Inv(btot), Wk(btot);
            DBuf<int32_t> piv(std::max<int64_t>(4 * maxr_rep * (int64_t)(q1 - q0), 1));
            std::vector<InvDesc> jobs;
            int64_t bo = 0;
            for (size_t q = q0; q < q1; ++q) {
                const int s = reps[q];
                const int r = (int)full.r[s];
                launch_full_block(r, Sg.p + soff[s], full.cptr.p + goff[s], full.ccol.p, full.cval64.p, Bm.p + bo,
                                  st);
                jobs.push_back(
                    {2 * r, Bm.p + bo, Wk.p + bo, Inv.p + bo, piv.p + 4 * maxr_rep * (int64_t)(q - q0), 2 * r});
                bo += 4 * (int64_t)r * r;
            }
            launch_invert_blocked(jobs, status.p, st);
            bo = 0;
            for (size_t q = q0; q < q1; ++q) {
                const int s = reps[q];
                const int r = (int)full.r[s];
                launch_full_extract(r, Inv.p + bo, full.m64.p + 2 * moff[s], full.m32.p + 2 * moff[s], st);
                bo += 4 * (int64_t)r * r;
            }
            THM_HIP(hipStreamSynchronize(st));
            if (std::getenv("THM_PROGRESS"))
                std::fprintf(stderr, "[thm] complete inverse: inverted %zu of %zu boundary matrices, %.1f s\n", q1,
                             reps.size(), (now_ms() - t0) * 1e-3);
            q0 = q1;
        }
        int32_t hs = 0;
        THM_HIP(hipMemcpyAsync(&hs, status.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        THM_HIP(hipStreamSynchronize(st));
        if (hs) fail(THM_ESINGULAR, "I + i C_G S_G is singular");
    }
    const int64_t gt = std::max<int64_t>(goff[ns], 1);
    full.u64.alloc(2 * gt);
    full.u32.alloc(2 * gt);
    full.part64.alloc(2 * gt * std::max(d.nchmax, 1));
    full.part32.alloc(2 * gt * std::max(d.nchmax, 1));
    full.w64.alloc(K.B.Ltot);
    full.y64.alloc(K.B.Ltot);
    full.w32.alloc(K.B.Ltot);
    full.y32.alloc(K.B.Ltot);
    THM_HIP(hipMemsetAsync(full.w64.p, 0, sizeof(double) * full.w64.n, st));
    THM_HIP(hipMemsetAsync(full.w32.p, 0, sizeof(float) * full.w32.n, st));
    full.neg1.upload(std::vector<double>(ns, -1.0), st);
    full.bytes = mtot * (16 + 8);
    THM_HIP(hipStreamSynchronize(st));
    full.setup_ms = now_ms() - t0;
    full.ready = true;
}

void Ctx::ensure_xi(bool f32) {
    if (f32 && !xi32.n) {
        xi32.alloc(2 * std::max<int64_t>(xi_total, 1));
        THM_HIP(hipMemsetAsync(xi32.p, 0, sizeof(float) * xi32.n, st));
    }
    if (!f32 && !xi64.n) {
        xi64.alloc(2 * std::max<int64_t>(xi_total, 1));
        THM_HIP(hipMemsetAsync(xi64.p, 0, sizeof(double) * xi64.n, st));
    }
}

KOps<double> Ctx::ops64(float csign, bool with_prec, int pkind) {
    if (with_prec) build_prec();
    if (with_prec && pkind == 1) build_full();
    KOps<double> o;
    o.apply = [this, csign](const double *x, double *y, const double *b, const int32_t *mask) {
        spmv<double>(lpr64, mask, x, y, b, csign);
    };
    if (with_prec && pkind == 0 && lpr64 == SPMV_SELL_GROUP_IL && spmv_shared) {
        ensure_xi(false);
        o.prec_i = [this](const double *x, double *y, const int32_t *mask) {
            const IlOut<double> il{sgroups.p, &ilsched, ngroups, xi64.p};
            launch_prec_apply<double>(P, P.d64.p, K.B.off.p, ns, mask, x, y, ws64.p, ys64.p, tw64.p, st, &il);
        };
        o.apply_i = [this, csign](double *y, const int32_t *mask) {
            launch_spmv_group_i<double>(mat64.p, K.B.off.p, sgroups.p, gsched, ngroups, mask, xi64.p, y, csign, st);
        };
    }
    o.prec = [this, csign, pkind](const double *x, double *y, const int32_t *mask) {
        if (!prec_ready) fail(THM_EINVAL, "preconditioner used before it was built");
        launch_prec_apply<double>(P, P.d64.p, K.B.off.p, ns, mask, x, y, ws64.p, ys64.p, tw64.p, st);
        if (pkind == 1) {
            // y -= K^{-1} P^T M^{-1} (+-i C_G y_G)
            launch_full_correct<double>(full.d, ns, mask, K.B.off.p, csign < 0 ? 1 : 0, y, full.u64.p,
                                        full.part64.p, full.w64.p, st);
            launch_prec_apply<double>(P, P.d64.p, K.B.off.p, ns, mask, full.w64.p, full.y64.p, ws64.p, ys64.p,
                                      tw64.p, st);
            launch_axpy<double, double>(K.B, mask, full.neg1.p, full.y64.p, y, st);
        }
    };
    o.graphable = true;
    o.owner = this;
    o.csign = csign;
    o.pkind = pkind;
    return o;
}

KOps<float> Ctx::ops32(float csign, bool with_prec, int pkind) {
    if (!x32.n) {
        x32.alloc(K.B.Ltot);
        b32.alloc(K.B.Ltot);
        THM_HIP(hipMemsetAsync(x32.p, 0, sizeof(float) * x32.n, st));
        THM_HIP(hipMemsetAsync(b32.p, 0, sizeof(float) * b32.n, st));
    }
    if (with_prec) {
        build_prec();
        if (!ws32.n) {
            ws32.alloc(P.Stot);
            ys32.alloc(P.Stot);
            tw32.alloc(2 * P.Ttot);
            THM_HIP(hipMemsetAsync(ws32.p, 0, sizeof(float) * ws32.n, st));
            THM_HIP(hipMemsetAsync(ys32.p, 0, sizeof(float) * ys32.n, st));
        }
    }
    KOps<float> o;
    o.apply = [this, csign](const float *x, float *y, const float *b, const int32_t *mask) {
        spmv<float>(lpr32, mask, x, y, b, csign);
    };
    if (with_prec && pkind == 1) build_full();
    o.prec = [this, csign, pkind](const float *x, float *y, const int32_t *mask) {
        prec32(pkind, csign, x, y, mask);
    };
    if (with_prec && pkind == 0 && lpr32 == SPMV_SELL_GROUP_IL && spmv_shared) {
        ensure_xi(true);
        o.prec_i = [this](const float *x, float *y, const int32_t *mask) {
            const IlOut<float> il{sgroups.p, &ilsched, ngroups, xi32.p};
            launch_prec_apply<float>(P, P.d32.p, K.B.off.p, ns, mask, x, y, ws32.p, ys32.p, tw32.p, st, &il);
        };
        o.apply_i = [this, csign](float *y, const int32_t *mask) {
            launch_spmv_group_i<float>(mat32.p, K.B.off.p, sgroups.p, gsched, ngroups, mask, xi32.p, y, csign, st);
        };
    }
    o.graphable = true;
    o.owner = this;
    o.csign = csign;
    o.pkind = pkind;
    return o;
}

void Ctx::prec32(int pkind, float csign, const float *x, float *y, const int32_t *mask) {
    if (!ws32.n) fail(THM_EINVAL, "preconditioner used before it was built");
    launch_prec_apply<float>(P, P.d32.p, K.B.off.p, ns, mask, x, y, ws32.p, ys32.p, tw32.p, st);
    if (pkind == 1) {
        // y -= K^{-1} P^T M^{-1} (+-i C_G y_G)
        launch_full_correct<float>(full.d, ns, mask, K.B.off.p, csign < 0 ? 1 : 0, y, full.u32.p, full.part32.p,
                                   full.w32.p, st);
        launch_prec_apply<float>(P, P.d32.p, K.B.off.p, ns, mask, full.w32.p, full.y32.p, ws32.p, ys32.p, tw32.p,
                                 st);
        launch_axpy<float, float>(K.B, mask, full.neg1.p, full.y32.p, y, st);
    }
}

KOps<double> Ctx::ops_mixed(float csign, int pk) {
    ops32(csign, true, pk);  // FP32 factor and work vectors (and the FP32 boundary correction)
    if (!mx32.n) {
        mx32.alloc(K.B.Ltot);
        my32.alloc(K.B.Ltot);
        THM_HIP(hipMemsetAsync(mx32.p, 0, sizeof(float) * mx32.n, st));
        THM_HIP(hipMemsetAsync(my32.p, 0, sizeof(float) * my32.n, st));
    }
    KOps<double> o;
    o.apply = [this, csign](const double *x, double *y, const double *b, const int32_t *mask) {
        spmv<double>(lpr64, mask, x, y, b, csign);
    };
    o.prec = [this, csign, pk](const double *x, double *y, const int32_t *mask) {
        launch_scale<double, float>(K.B, mask, nullptr, 0, x, mx32.p, nullptr, 0, nullptr, st);
        prec32(pk, csign, mx32.p, my32.p, mask);
        launch_scale<float, double>(K.B, mask, nullptr, 0, my32.p, y, nullptr, 0, nullptr, st);
    };
    o.graphable = true;
    o.owner = this;
    o.csign = csign;
    o.pkind = 2 + pk;
    return o;
}

void Ctx::solve(const thm_solve_opts &o, float csign, const int32_t *mask, std::vector<int> &iters,
                std::vector<int> &refines, std::vector<double> &resid) {
    if (!mask) mask = mask_all.p;
    last_fb.assign(ns, 0);
    last_ir.assign(ns, 0);
    iters.assign(ns, 0);
    refines.assign(ns, 0);
    resid.assign(ns, 0.0);
    std::vector<int32_t> hi(ns);
    std::vector<double> hr(ns);
    GmresParams gp;
    gp.rtol = o.rtol;
    gp.max_iter = o.max_iter;
    gp.orth = o.orth;
    gp.use_graph = o.use_graph != 0;
    gp.cplx = o.krylov == THM_KRYLOV_COMPLEX ? 1 : 0;
    const int pk = o.precond == THM_PREC_FULL ? 1 : 0;
    if (o.precision == THM_FP64) {
        gmres_run<double>(K, ops64(csign, true, pk), b64.p, x64.p, mask, gp, st);
        THM_HIP(hipMemcpyAsync(hi.data(), K.iters.p, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st));
        THM_HIP(hipMemcpyAsync(hr.data(), K.resid.p, sizeof(double) * ns, hipMemcpyDeviceToHost, st));
        THM_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < ns; ++i) {
            iters[i] = hi[i];
            resid[i] = hr[i];
        }
        return;
    }
    // FP32 inner GMRES inside FP64 iterative refinement
    KOps<double> A64 = ops64(csign, true, pk);
    KOps<float> A32 = ops32(csign, true, pk);
    launch_norm2<double>(K.B, mask, b64.p, K.part.p, st);
    launch_norm_finish(K.B, K.part.p, mask, bnorm64.p, nullptr, 0.0, nullptr, nullptr, st);
    THM_HIP(hipMemcpyAsync(run_ir.p, mask, sizeof(int32_t) * ns, hipMemcpyDeviceToDevice, st));
    // FP32 inner solves: one GMRES cycle each (stopped by the FP64 Givens estimate);
    // accuracy comes from the FP64 refinement loop, not from the FP32 residual.
    // Safeguard: a step that does not at least halve a system's FP64 residual (the FP32
    // factor is too inaccurate for that system's K, e.g. near a resonance) is undone and
    // the system is finished by GMRES-IR (FP64 GMRES preconditioned by the FP32 factor) from
    // its current iterate, as is every system still running when max_refine steps are spent;
    // FP64 GMRES with the FP64 factor is the last resort if that misses rtol.
    GmresParams ip = gp;
    ip.rtol = o.ir_inner_rtol;
    ip.max_iter = std::min(o.max_iter, K.m);
    std::vector<double> prev(ns, HUGE_VAL), rn_last(ns, 0.0), hrn(ns);
    std::vector<int32_t> stepped(ns, 0), fb(ns, 0), undo(ns, 0);
    auto upload_flags = [&](DBuf<int32_t> &dst, const std::vector<int32_t> &h) {
        THM_HIP(hipMemcpyAsync(dst.p, h.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, st));
    };
    if (!ir_aux.n) ir_aux.alloc(ns);
    if (!ir_scal.n) ir_scal.alloc(ns);
    const bool classic = o.ir_mode != THM_IR_GMRES;
    std::vector<int32_t> &sticky = ir_sticky[pk];
    if (sticky.size() != (size_t)ns) sticky.assign(ns, 0);
    {
        // GMRES-IR from the start for every system (THM_IR_GMRES) or for the systems whose
        // classical step has already failed to contract in this context
        std::vector<int32_t> hm(ns);
        THM_HIP(hipMemcpyAsync(hm.data(), mask, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st));
        THM_HIP(hipStreamSynchronize(st));
        bool any_sticky = false;
        for (int i = 0; i < ns; ++i) {
            fb[i] = hm[i] && (!classic || sticky[i]);
            any_sticky = any_sticky || fb[i];
            if (fb[i]) hm[i] = 0;
        }
        if (classic && any_sticky) upload_flags(run_ir, hm);
    }
    for (int it = 0; classic; ++it) {
        A64.apply(x64.p, r64.p, b64.p, run_ir.p);
        launch_norm2<double>(K.B, run_ir.p, r64.p, K.part.p, st);
        launch_norm_finish(K.B, K.part.p, run_ir.p, rnorm.p, bnorm64.p, o.rtol, resid64.p, run_ir.p, st);
        THM_HIP(hipMemcpyAsync(hi.data(), run_ir.p, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st));
        THM_HIP(hipMemcpyAsync(hr.data(), resid64.p, sizeof(double) * ns, hipMemcpyDeviceToHost, st));
        THM_HIP(hipMemcpyAsync(hrn.data(), rnorm.p, sizeof(double) * ns, hipMemcpyDeviceToHost, st));
        THM_HIP(hipStreamSynchronize(st));
        bool any_undo = false;
        for (int i = 0; i < ns; ++i) {
            undo[i] = stepped[i] && !(hr[i] <= 0.5 * prev[i]) && hr[i] > o.rtol;
            if (undo[i]) {
                any_undo = true;
                fb[i] = 1;
                sticky[i] = 1;
                hi[i] = 0;
                hr[i] = prev[i];
            }
            stepped[i] = 0;
        }
        if (any_undo) {
            // x -= (previous residual norm) * (previous FP32 correction), still in x32
            std::vector<double> neg(ns);
            for (int i = 0; i < ns; ++i) neg[i] = -rn_last[i];
            THM_HIP(hipMemcpyAsync(ir_scal.p, neg.data(), sizeof(double) * ns, hipMemcpyHostToDevice, st));
            upload_flags(ir_aux, undo);
            launch_axpy<double, float>(K.B, ir_aux.p, ir_scal.p, x32.p, x64.p, st);
            upload_flags(run_ir, hi);
        }
        bool any = false;
        for (int i = 0; i < ns; ++i) any = any || hi[i];
        if (!any) break;
        if (it >= o.max_refine) {
            for (int i = 0; i < ns; ++i)
                if (hi[i]) fb[i] = 1;
            break;
        }
        double worst = 0.0;
        for (int i = 0; i < ns; ++i)
            if (hi[i]) {
                refines[i]++;
                worst = std::max(worst, hr[i]);
                prev[i] = hr[i];
                rn_last[i] = hrn[i];
                stepped[i] = 1;
            }
        // the inner FP32 solve only has to gain the remaining factor (with margin),
        // but never goes below what FP32 Arnoldi resolves
        ip.rtol = std::max(o.ir_inner_rtol, 0.3 * o.rtol / std::max(worst, 1e-300));
        launch_scale<double, float>(K.B, run_ir.p, rnorm.p, 1, r64.p, b32.p, nullptr, 0, nullptr, st);
        THM_HIP(hipMemsetAsync(x32.p, 0, sizeof(float) * x32.n, st));
        gmres_run<float>(K, A32, b32.p, x32.p, run_ir.p, ip, st);
        launch_axpy<double, float>(K.B, run_ir.p, rnorm.p, x32.p, x64.p, st);
        THM_HIP(hipMemcpyAsync(hi.data(), K.iters.p, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st));
        THM_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < ns; ++i) iters[i] += hi[i];
    }
    if (classic) {
        THM_HIP(hipMemcpyAsync(hr.data(), resid64.p, sizeof(double) * ns, hipMemcpyDeviceToHost, st));
        THM_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < ns; ++i) resid[i] = hr[i];
    }
    bool any_fb = false;
    for (int i = 0; i < ns; ++i) any_fb = any_fb || fb[i];
    if (any_fb) {
        // GMRES-based refinement (Carson & Higham, SIAM J. Sci. Comput. 40 (2018)): where a
        // classical step with an FP32 inner solve did not contract, the correction is solved by
        // GMRES in FP64 (FP64 operator, basis, Hessenberg) with the FP32 factor as the
        // preconditioner, from the current iterate.  The FP32 factor only slows convergence
        // there, it no longer limits the attainable accuracy.  It runs one restart cycle at a
        // time, and a cycle must at least halve a system's FP64 residual (the same rule as a
        // classical step); a system that stalls (its FP32 factor too far from K^{-1}, e.g. near
        // a resonance) is finished with the FP64 factor below.
        KOps<double> AM = ops_mixed(csign, pk);
        GmresParams cp = gp;
        cp.max_iter = K.m;
        std::vector<int32_t> in_ir(fb);
        std::vector<double> prev_ir(ns, HUGE_VAL);  // no bar on a system's first cycle
        int used = 0;
        for (;;) {
            bool any_ir = false;
            for (int i = 0; i < ns; ++i) any_ir = any_ir || in_ir[i];
            if (!any_ir) break;
            if (used >= o.max_iter) {
                for (int i = 0; i < ns; ++i) in_ir[i] = 0;  // fb stays set: FP64 below
                break;
            }
            upload_flags(ir_aux, in_ir);
            gmres_run<double>(K, AM, b64.p, x64.p, ir_aux.p, cp, st);
            THM_HIP(hipMemcpyAsync(hi.data(), K.iters.p, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st));
            THM_HIP(hipMemcpyAsync(hr.data(), K.resid.p, sizeof(double) * ns, hipMemcpyDeviceToHost, st));
            THM_HIP(hipStreamSynchronize(st));
            int cyc = 0;
            for (int i = 0; i < ns; ++i) {
                if (!in_ir[i]) continue;
                iters[i] += hi[i];
                cyc = std::max(cyc, hi[i]);
                resid[i] = hr[i];
                last_ir[i] = 1;
                if (hr[i] <= o.rtol) {
                    in_ir[i] = 0;
                    fb[i] = 0;
                } else if (!(hr[i] <= 0.5 * prev_ir[i])) {
                    in_ir[i] = 0;  // stalled: FP64 below
                } else {
                    prev_ir[i] = hr[i];
                }
            }
            used += std::max(cyc, 1);
        }
        any_fb = false;
        for (int i = 0; i < ns; ++i) any_fb = any_fb || fb[i];
    }
    if (any_fb) {
        upload_flags(ir_aux, fb);
        gmres_run<double>(K, A64, b64.p, x64.p, ir_aux.p, gp, st);
        THM_HIP(hipMemcpyAsync(hi.data(), K.iters.p, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st));
        THM_HIP(hipMemcpyAsync(hr.data(), K.resid.p, sizeof(double) * ns, hipMemcpyDeviceToHost, st));
        THM_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < ns; ++i)
            if (fb[i]) {
                iters[i] += hi[i];
                resid[i] = hr[i];
                fp64_fallbacks++;
                last_fb[i] = 1;
            }
    }
}

double Ctx::time_bcr(int prec, int reps, double *bytes, int *launches) {
    build_prec();
    if (prec) ops32(1.f);
    hipEvent_t e0, e1;
    THM_HIP(hipEventCreate(&e0));
    THM_HIP(hipEventCreate(&e1));
    auto once = [&] {
        if (prec) launch_bcr_phases<float>(P, nullptr, ws32.p, ys32.p, st);
        else launch_bcr_phases<double>(P, nullptr, ws64.p, ys64.p, st);
    };
    once();
    THM_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) once();
    THM_HIP(hipEventRecord(e1, st));
    THM_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    THM_HIP(hipEventElapsedTime(&ms, e0, e1));
    THM_HIP(hipEventDestroy(e0));
    THM_HIP(hipEventDestroy(e1));
    double by = 0.0;
    for (double b : bcr_bytes[prec]) by += b;
    if (bytes) *bytes = by;
    if (launches) *launches = (int)P.phases.size();
    return ms / reps;
}

void Ctx::copy_in(int s, const double *src, double *slot) {
    THM_HIP(hipMemcpyAsync(slot + K.B.h_off[s], src, sizeof(double) * 2 * sys[s]->n, hipMemcpyDeviceToDevice, st));
}
void Ctx::copy_out(int s, const double *slot, double *dst) {
    THM_HIP(hipMemcpyAsync(dst, slot + K.B.h_off[s], sizeof(double) * 2 * sys[s]->n, hipMemcpyDeviceToDevice, st));
}

// ------------------------------------------------------------------ SpMV autotuner
// Picks the lanes-per-row of the CSR-vector SpMV for a batch by timing the candidates
// on the batch's own matrices.  Results are cached per (dim, degree, size bucket,
// batch size, precision) in-process and, if THM_TUNE_CACHE names a file, on disk
// as "key lpr" lines.
static std::mutex g_tune_mu;
static std::map<std::string, int> g_tune;
static bool g_tune_loaded = false;

static void tune_load() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *f = std::getenv("THM_TUNE_CACHE");
    if (!f) return;
    std::ifstream in(f);
    std::string k;
    int v;
    while (in >> k >> v) g_tune[k] = v;
}

static void tune_store() {
    const char *f = std::getenv("THM_TUNE_CACHE");
    if (!f) return;
    std::ofstream out(f);
    for (auto &kv : g_tune) out << kv.first << " " << kv.second << "\n";
}

void Ctx::autotune() {
    std::vector<int> cand = {21, 41, 81, 161, 321, 24, 44, 84, 164, 324, SPMV_SELL};
    if (spmv_shared) cand.push_back(SPMV_SELL_GROUP);
    for (int c : cand)
        if (c != SPMV_SELL_GROUP) K.B.spmv_sched(c, st);
    int64_t nnz = 0, nrows = 0;
    for (thm_system *s : sys) {
        nnz += (int64_t)s->K.col.size();
        nrows += s->n;
    }
    const thm_system &s0 = *sys[0];
    int nb = 0;
    while ((int64_t(1) << (nb + 1)) <= nrows) ++nb;
    char key64[128], key32[128];
    std::snprintf(key64, sizeof key64, "gfx950:d%d:p%d:n%d:b%d:g%d:fp64", s0.topo.dim, s0.topo.p, nb, ns, ngroups);
    std::snprintf(key32, sizeof key32, "gfx950:d%d:p%d:n%d:b%d:g%d:fp32", s0.topo.dim, s0.topo.p, nb, ns, ngroups);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load();
        auto a = g_tune.find(key64), b = g_tune.find(key32);
        if (a != g_tune.end() && b != g_tune.end()) {
            lpr64 = a->second;
            lpr32 = b->second;
            return;
        }
    }
    (void)nnz;
    hipEvent_t e0, e1;
    THM_HIP(hipEventCreate(&e0));
    THM_HIP(hipEventCreate(&e1));
    auto time_it = [&](auto launch) {
        launch();
        THM_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < 3; ++r) launch();
        THM_HIP(hipEventRecord(e1, st));
        THM_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        THM_HIP(hipEventElapsedTime(&ms, e0, e1));
        return ms;
    };
    float best = 1e30f;
    for (int c : cand) {
        const float ms = time_it([&] { spmv<double>(c, nullptr, x64.p, r64.p, nullptr, 1.f); });
        if (ms < best) { best = ms; lpr64 = c; }
    }
    ops32(1.f, false);
    best = 1e30f;
    for (int c : cand) {
        const float ms = time_it([&] { spmv<float>(c, nullptr, x32.p, b32.p, nullptr, 1.f); });
        if (ms < best) { best = ms; lpr32 = c; }
    }
    THM_HIP(hipEventDestroy(e0));
    THM_HIP(hipEventDestroy(e1));
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key64] = lpr64;
    g_tune[key32] = lpr32;
    tune_store();
}

}  // namespace thm
