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
    B.init(n, m + 2, st);
    const int ns = B.ns;
    H.alloc((size_t)ns * (m + 1) * m);
    cs.alloc((size_t)ns * m);
    sn.alloc((size_t)ns * m);
    g.alloc((size_t)ns * (m + 1));
    y.alloc((size_t)ns * (m + 1));
    hcol.alloc((size_t)ns * (m + 1));
    hcol2.alloc((size_t)ns * (m + 1));
    for (DBuf<double> *b : {&hnext, &bnorm, &beta, &resid, &est}) b->alloc(ns);
    part.alloc((size_t)std::max(1, B.vs.nblocks) * B.maxcols);
    for (DBuf<int32_t> *b : {&running, &active, &jcnt, &iters}) b->alloc(ns);
    if (!pinned) THM_HIP(hipHostMalloc((void **)&pinned, sizeof(int32_t) * 2 * std::max(ns, 1)));
    else {
        (void)hipHostFree(pinned);
        THM_HIP(hipHostMalloc((void **)&pinned, sizeof(int32_t) * 2 * std::max(ns, 1)));
    }
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
    for (auto &s : slots) {
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

template <class T>
static void arnoldi_step(Krylov &K, const KOps<T> &ops, const GmresParams &p, hipStream_t st) {
    Batch &B = K.B;
    const int m = K.m;
    T *V = K.V<T>(), *w = K.w<T>(), *z = K.z<T>(), *cur = K.cur<T>();
    int32_t *act = K.active.p;
    ops.prec(cur, z, act);
    ops.apply(z, w, nullptr, act);
    launch_dots<T>(B, act, K.jcnt.p, V, B.Ltot, w, K.part.p, st);
    launch_reduce_cols(B, act, K.jcnt.p, 0, K.part.p, K.hcol.p, m + 1, 0, st);
    launch_cgs_update<T>(B, act, K.jcnt.p, V, B.Ltot, w, K.hcol.p, m + 1, K.part.p, st);
    if (p.orth == THM_ORTH_CGS2) {
        launch_dots<T>(B, act, K.jcnt.p, V, B.Ltot, w, K.part.p, st);
        launch_reduce_cols(B, act, K.jcnt.p, 0, K.part.p, K.hcol2.p, m + 1, 0, st);
        launch_reduce_cols(B, act, K.jcnt.p, 0, K.part.p, K.hcol.p, m + 1, 1, st);
        launch_cgs_update<T>(B, act, K.jcnt.p, V, B.Ltot, w, K.hcol2.p, m + 1, K.part.p, st);
    }
    launch_arnoldi_finish(B, K.part.p, act, K.jcnt.p, K.hcol.p, m + 1, K.H.p, K.cs.p, K.sn.p, K.g.p, K.hnext.p,
                          K.bnorm.p, p.rtol, m, K.iters.p, p.max_iter, K.est.p, st);
    launch_scale<T, T>(B, act, K.hnext.p, 1, w, V, K.jcnt.p, B.Ltot, cur, st);
}

template <class T>
static hipGraphExec_t step_graph(Krylov &K, const KOps<T> &ops, const GmresParams &p, hipStream_t st) {
    const int key = TypeKey<T>::v * 2 + (ops.csign < 0 ? 1 : 0);
    Krylov::GraphSlot &s = K.slots[key];
    if (s.exec && s.owner == ops.owner && s.orth == p.orth && s.rtol == p.rtol && s.max_iter == p.max_iter)
        return s.exec;
    if (s.exec) (void)hipGraphExecDestroy(s.exec);
    if (s.graph) (void)hipGraphDestroy(s.graph);
    s = Krylov::GraphSlot{};
    THM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
        arnoldi_step<T>(K, ops, p, st);
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
    s.csign = ops.csign;
    s.key_T = TypeKey<T>::v;
    return s.exec;
}

static bool any_set(const int32_t *h, int ns) {
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
    T *V = K.V<T>(), *w = K.w<T>(), *z = K.z<T>(), *cur = K.cur<T>();
    launch_norm2<T>(B, mask_in, b, K.part.p, st);
    launch_norm_finish(B, K.part.p, mask_in, K.bnorm.p, nullptr, 0.0, nullptr, nullptr, st);
    THM_HIP(hipMemcpyAsync(K.running.p, mask_in, sizeof(int32_t) * ns, hipMemcpyDeviceToDevice, st));
    THM_HIP(hipMemsetAsync(K.iters.p, 0, sizeof(int32_t) * ns, st));
    const bool graph = p.use_graph && ops.graphable;
    hipGraphExec_t exec = graph ? step_graph<T>(K, ops, p, st) : nullptr;
    int32_t *hflag[2] = {K.pinned, K.pinned + ns};
    for (;;) {
        ops.apply(x, w, b, K.running.p);
        launch_norm2<T>(B, K.running.p, w, K.part.p, st);
        launch_cycle_start(B, K.part.p, K.running.p, K.active.p, K.jcnt.p, K.bnorm.p, p.rtol, K.g.p, m, K.beta.p,
                           K.resid.p, K.iters.p, p.max_iter, st);
        THM_HIP(hipMemcpyAsync(hflag[0], K.running.p, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st));
        THM_HIP(hipStreamSynchronize(st));
        if (!any_set(hflag[0], ns)) break;
        launch_scale<T, T>(B, K.active.p, K.beta.p, 1, w, V, K.jcnt.p, B.Ltot, cur, st);
        // Arnoldi steps; the host checks step j-1's flags while step j runs.
        for (int step = 0; step < m; ++step) {
            if (exec) THM_HIP(hipGraphLaunch(exec, st));
            else arnoldi_step<T>(K, ops, p, st);
            const int sl = step & 1;
            THM_HIP(hipMemcpyAsync(hflag[sl], K.active.p, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st));
            THM_HIP(hipEventRecord(K.ev[sl], st));
            if (step > 0) {
                THM_HIP(hipEventSynchronize(K.ev[sl ^ 1]));
                if (!any_set(hflag[sl ^ 1], ns)) break;
            }
        }
        launch_hsolve(B, K.running.p, K.jcnt.p, K.H.p, K.g.p, K.y.p, m, st);
        launch_lincomb<T>(B, K.running.p, K.jcnt.p, V, B.Ltot, K.y.p, m + 1, cur, st);
        ops.prec(cur, z, K.running.p);
        launch_axpy<T, T>(B, K.running.p, nullptr, z, x, st);
    }
}

template void gmres_run<double>(Krylov &, const KOps<double> &, const double *, double *, const int32_t *,
                                const GmresParams &, hipStream_t);
template void gmres_run<float>(Krylov &, const KOps<float> &, const float *, float *, const int32_t *,
                               const GmresParams &, hipStream_t);

// ------------------------------------------------------------------ preconditioner setup
void setup_precond(const std::vector<thm_system *> &all, hipStream_t st) {
    std::vector<thm_system *> sys;
    for (thm_system *s : all)
        if (!s->prec_ready) sys.push_back(s);
    if (sys.empty()) return;
    const double t0 = now_ms();
    DBuf<int32_t> status(1);
    THM_HIP(hipMemsetAsync(status.p, 0, sizeof(int32_t), st));
    std::vector<DBuf<double>> work0(sys.size()), work1(sys.size()), btmp(sys.size());
    std::vector<DBuf<int32_t>> piv(sys.size());
    int maxL = 0;
    for (size_t i = 0; i < sys.size(); ++i) {
        thm_system &S = *sys[i];
        const Layering &L = S.L;
        const Topo &t = S.topo;
        S.Lskel_dof.upload(L.skel_dof, st);
        S.Ldof_pos.upload(L.dof_pos, st);
        S.Lcond_ptr.upload(L.cond_ptr, st);
        S.Lcond_cell.upload(L.cond_cell, st);
        S.Lcond_loc.upload(L.cond_loc, st);
        S.Lbsize.upload(L.bsize, st);
        S.Lboff.upload(L.boff, st);
        S.Lsinv_off.upload(L.sinv_off, st);
        S.Llf_off.upload(L.lf_off, st);
        const int ne = t.n_loc - t.n_int;
        S.kiinv.alloc((size_t)t.n_cells * t.n_int * t.n_int);
        S.F.alloc((size_t)t.n_cells * ne * t.n_int);
        DBuf<double> kcond((size_t)t.n_cells * ne * ne);
        launch_condense((int)t.n_cells, t.n_loc, t.n_int, S.kel.p, S.cell_dofs.p, S.dir_d.p, S.kiinv.p, S.F.p, kcond.p,
                        status.p, st);
        S.sinv.alloc(L.sinv_total);
        S.lf.alloc(std::max<int64_t>(L.lf_total, 1));
        S.lft.alloc(std::max<int64_t>(L.lf_total, 1));
        launch_fill(S.sinv.p, L.sinv_total, 0.0, st);
        launch_fill(S.lf.p, L.lf_total, 0.0, st);
        {
            DBuf<int64_t> ti;
            DBuf<int32_t> tk, tp, ts;
            ti.upload(L.tgt_index, st);
            tk.upload(L.tgt_kind, st);
            tp.upload(L.tgt_ptr, st);
            ts.upload(L.tgt_src, st);
            launch_tgt_gather((int64_t)L.tgt_index.size(), ti.p, tk.p, tp.p, ts.p, kcond.p, S.sinv.p, S.lf.p, st);
            THM_HIP(hipStreamSynchronize(st));
        }
        launch_dir_identity(L.n_skel, S.Lskel_dof.p, S.dir_d.p, S.Lboff.p, S.Lsinv_off.p, S.Lbsize.p, L.nlayers,
                            S.sinv.p, st);
        int bmax = 0;
        for (int b : L.bsize) bmax = std::max(bmax, b);
        work0[i].alloc((size_t)bmax * bmax);
        work1[i].alloc((size_t)bmax * bmax);
        btmp[i].alloc((size_t)bmax * bmax);
        piv[i].alloc((size_t)2 * bmax);
        maxL = std::max(maxL, L.nlayers);
        THM_HIP(hipStreamSynchronize(st));
    }
    DBuf<GemmDesc> gscr;
    DBuf<InvDesc> iscr;
    Sched gsched;
    for (int k = 0; k < maxL; ++k) {
        std::vector<GemmDesc> g1, g2;
        std::vector<InvDesc> inv;
        for (size_t i = 0; i < sys.size(); ++i) {
            thm_system &S = *sys[i];
            const Layering &L = S.L;
            if (k >= L.nlayers) continue;
            const int bk = L.bsize[k];
            double *sk = S.sinv.p + L.sinv_off[k];
            THM_HIP(hipMemcpyAsync(work0[i].p, sk, sizeof(double) * bk * bk, hipMemcpyDeviceToDevice, st));
            if (k > 0) {
                const int bp = L.bsize[k - 1];
                double *lfk = S.lf.p + L.lf_off[k];
                THM_HIP(hipMemcpyAsync(btmp[i].p, lfk, sizeof(double) * bk * bp, hipMemcpyDeviceToDevice, st));
                // Lf_k = B_k S_{k-1}^{-1}
                g1.push_back({bk, bp, bp, 0, 0, btmp[i].p, S.sinv.p + L.sinv_off[k - 1], lfk, bp, bp, bp, 1.0, 0.0});
                // S_k = A_k - Lf_k B_k^T
                g2.push_back({bk, bk, bp, 0, 1, lfk, btmp[i].p, work0[i].p, bp, bp, bk, -1.0, 1.0});
            }
            inv.push_back({bk, work0[i].p, work1[i].p, sk, piv[i].p});
        }
        launch_gemm_batched(g1, st, gscr, gsched);
        THM_HIP(hipStreamSynchronize(st));
        launch_gemm_batched(g2, st, gscr, gsched);
        THM_HIP(hipStreamSynchronize(st));
        launch_invert_batched(inv, status.p, st, iscr);
    }
    for (thm_system *sp : sys) {
        thm_system &S = *sp;
        const Layering &L = S.L;
        for (int k = 1; k < L.nlayers; ++k)
            launch_transpose(S.lf.p + L.lf_off[k], L.bsize[k], L.bsize[k - 1], S.lft.p + L.lf_off[k], st);
        S.sinv32.alloc(S.sinv.n);
        S.lf32.alloc(S.lf.n);
        S.lft32.alloc(S.lft.n);
        S.kiinv32.alloc(std::max<size_t>(S.kiinv.n, 1));
        S.F32.alloc(std::max<size_t>(S.F.n, 1));
        launch_convert(S.sinv.p, S.sinv32.p, S.sinv.n, st);
        launch_convert(S.lf.p, S.lf32.p, S.lf.n, st);
        launch_convert(S.lft.p, S.lft32.p, S.lft.n, st);
        launch_convert(S.kiinv.p, S.kiinv32.p, S.kiinv.n, st);
        launch_convert(S.F.p, S.F32.p, S.F.n, st);
    }
    int32_t hs = 0;
    THM_HIP(hipMemcpyAsync(&hs, status.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    THM_HIP(hipStreamSynchronize(st));
    if (hs) fail(THM_ESINGULAR, "zero or non-finite pivot while factorising the block preconditioner");
    const double dt = now_ms() - t0;
    for (thm_system *s : sys) {
        s->prec_ready = true;
        s->prec_setup_ms = dt;
    }
}

// ------------------------------------------------------------------ batched context
void Ctx::build(const std::vector<thm_system *> &s, int m, hipStream_t stream) {
    sys = s;
    ns = (int)s.size();
    st = stream;
    setup_precond(sys, st);
    std::vector<int64_t> n(ns), nsk(ns);
    for (int i = 0; i < ns; ++i) {
        n[i] = sys[i]->n;
        nsk[i] = sys[i]->L.n_skel;
    }
    K.init(n, m, st);
    std::vector<MatDesc> h64(ns), h32(ns);
    std::vector<const uint8_t *> hd(ns);
    std::vector<PrecDesc> p64(ns), p32(ns);
    std::vector<int64_t> soff(ns);
    int64_t so = 0;
    int maxL = 0;
    for (int i = 0; i < ns; ++i) {
        thm_system &S = *sys[i];
        h64[i] = {S.n, S.k_rowptr.p, S.k_col.p, S.kval.p, S.c_rowptr.p, S.c_col.p, S.cval.p};
        h32[i] = {S.n, S.k_rowptr.p, S.k_col.p, S.kval32.p, S.c_rowptr.p, S.c_col.p, S.cval32.p};
        hd[i] = S.dir_d.p;
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
        d.cell_dofs = S.cell_dofs.p;
        d.skel_dof = S.Lskel_dof.p;
        d.dof_pos = S.Ldof_pos.p;
        d.cond_ptr = S.Lcond_ptr.p;
        d.cond_cell = S.Lcond_cell.p;
        d.cond_loc = S.Lcond_loc.p;
        d.boff = S.Lboff.p;
        d.sinv_off = S.Lsinv_off.p;
        d.lf_off = S.Llf_off.p;
        d.bsize = S.Lbsize.p;
        p32[i] = d;
        d.sinv = S.sinv.p;
        d.lf = S.lf.p;
        d.lft = S.lft.p;
        d.kiinv = S.kiinv.p;
        d.F = S.F.p;
        p64[i] = d;
        p32[i].sinv = S.sinv32.p;
        p32[i].lf = S.lf32.p;
        p32[i].lft = S.lft32.p;
        p32[i].kiinv = S.kiinv32.p;
        p32[i].F = S.F32.p;
        soff[i] = so;
        so += 2 * nsk[i];
        so = (so + 63) & ~int64_t(63);
        maxL = std::max(maxL, S.L.nlayers);
    }
    mat64.upload(h64, st);
    mat32.upload(h32, st);
    dirs.upload(hd, st);
    P.ns = ns;
    P.maxlayers = maxL;
    P.d64.upload(p64, st);
    P.d32.upload(p32, st);
    P.soff.upload(soff, st);
    P.Stot = std::max<int64_t>(so, 64);
    P.skel.build(nsk, 256, st);
    P.skel_rows.build(nsk, 4, st);
    P.dofs.build(n, 256, st);
    P.fwd.clear();
    P.bwd.clear();
    P.fwd.resize(maxL);
    P.bwd.resize(maxL);
    for (int k = 0; k < maxL; ++k) {
        std::vector<int64_t> rf(ns, 0), rb(ns, 0);
        for (int i = 0; i < ns; ++i) {
            const Layering &L = sys[i]->L;
            if (k >= 1 && k < L.nlayers) rf[i] = L.bsize[k];
            if (k <= L.nlayers - 2) rb[i] = L.bsize[k];
        }
        P.fwd[k].build(rf, 4, st);
        P.bwd[k].build(rb, 4, st);
    }
    x64.alloc(K.B.Ltot);
    b64.alloc(K.B.Ltot);
    r64.alloc(K.B.Ltot);
    ws64.alloc(P.Stot);
    ys64.alloc(P.Stot);
    THM_HIP(hipMemsetAsync(x64.p, 0, sizeof(double) * x64.n, st));
    THM_HIP(hipMemsetAsync(b64.p, 0, sizeof(double) * b64.n, st));
    THM_HIP(hipMemsetAsync(r64.p, 0, sizeof(double) * r64.n, st));
    THM_HIP(hipMemsetAsync(ws64.p, 0, sizeof(double) * ws64.n, st));
    THM_HIP(hipMemsetAsync(ys64.p, 0, sizeof(double) * ys64.n, st));
    mask_all.upload(std::vector<int32_t>(ns, 1), st);
    run_ir.alloc(ns);
    rnorm.alloc(ns);
    bnorm64.alloc(ns);
    resid64.alloc(ns);
    THM_HIP(hipStreamSynchronize(st));
    autotune();
}

KOps<double> Ctx::ops64(float csign) {
    KOps<double> o;
    o.apply = [this, csign](const double *x, double *y, const double *b, const int32_t *mask) {
        const Sched &sc = K.B.spmv_sched(lpr64, st);
        launch_spmv<double>(lpr64, mat64.p, K.B.off.p, sc, ns, mask, x, y, b, csign, st);
    };
    o.prec = [this](const double *x, double *y, const int32_t *mask) {
        launch_prec_apply<double>(P, P.d64.p, K.B.off.p, ns, mask, x, y, ws64.p, ys64.p, st);
    };
    o.graphable = true;
    o.owner = this;
    o.csign = csign;
    return o;
}

KOps<float> Ctx::ops32(float csign) {
    if (!ws32.n) {
        ws32.alloc(P.Stot);
        ys32.alloc(P.Stot);
        x32.alloc(K.B.Ltot);
        b32.alloc(K.B.Ltot);
        THM_HIP(hipMemsetAsync(ws32.p, 0, sizeof(float) * ws32.n, st));
        THM_HIP(hipMemsetAsync(ys32.p, 0, sizeof(float) * ys32.n, st));
        THM_HIP(hipMemsetAsync(x32.p, 0, sizeof(float) * x32.n, st));
        THM_HIP(hipMemsetAsync(b32.p, 0, sizeof(float) * b32.n, st));
    }
    KOps<float> o;
    o.apply = [this, csign](const float *x, float *y, const float *b, const int32_t *mask) {
        const Sched &sc = K.B.spmv_sched(lpr32, st);
        launch_spmv<float>(lpr32, mat32.p, K.B.off.p, sc, ns, mask, x, y, b, csign, st);
    };
    o.prec = [this](const float *x, float *y, const int32_t *mask) {
        launch_prec_apply<float>(P, P.d32.p, K.B.off.p, ns, mask, x, y, ws32.p, ys32.p, st);
    };
    o.graphable = true;
    o.owner = this;
    o.csign = csign;
    return o;
}

void Ctx::solve(const thm_solve_opts &o, float csign, const int32_t *mask, std::vector<int> &iters,
                std::vector<int> &refines, std::vector<double> &resid) {
    if (!mask) mask = mask_all.p;
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
    if (o.precision == THM_FP64) {
        gmres_run<double>(K, ops64(csign), b64.p, x64.p, mask, gp, st);
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
    KOps<double> A64 = ops64(csign);
    KOps<float> A32 = ops32(csign);
    launch_norm2<double>(K.B, mask, b64.p, K.part.p, st);
    launch_norm_finish(K.B, K.part.p, mask, bnorm64.p, nullptr, 0.0, nullptr, nullptr, st);
    THM_HIP(hipMemcpyAsync(run_ir.p, mask, sizeof(int32_t) * ns, hipMemcpyDeviceToDevice, st));
    GmresParams ip = gp;
    ip.rtol = o.ir_inner_rtol;
    for (int it = 0;; ++it) {
        A64.apply(x64.p, r64.p, b64.p, run_ir.p);
        launch_norm2<double>(K.B, run_ir.p, r64.p, K.part.p, st);
        launch_norm_finish(K.B, K.part.p, run_ir.p, rnorm.p, bnorm64.p, o.rtol, resid64.p, run_ir.p, st);
        THM_HIP(hipMemcpyAsync(hi.data(), run_ir.p, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st));
        THM_HIP(hipStreamSynchronize(st));
        bool any = false;
        for (int i = 0; i < ns; ++i) any = any || hi[i];
        if (!any || it >= o.max_refine) break;
        for (int i = 0; i < ns; ++i)
            if (hi[i]) refines[i]++;
        launch_scale<double, float>(K.B, run_ir.p, rnorm.p, 1, r64.p, b32.p, nullptr, 0, nullptr, st);
        THM_HIP(hipMemsetAsync(x32.p, 0, sizeof(float) * x32.n, st));
        gmres_run<float>(K, A32, b32.p, x32.p, run_ir.p, ip, st);
        launch_axpy<double, float>(K.B, run_ir.p, rnorm.p, x32.p, x64.p, st);
        THM_HIP(hipMemcpyAsync(hi.data(), K.iters.p, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st));
        THM_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < ns; ++i) iters[i] += hi[i];
    }
    THM_HIP(hipMemcpyAsync(hr.data(), resid64.p, sizeof(double) * ns, hipMemcpyDeviceToHost, st));
    THM_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < ns; ++i) resid[i] = hr[i];
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
    const int cand[] = {2, 4, 8, 16, 32};
    for (int c : cand) K.B.spmv_sched(c, st);
    int64_t nnz = 0, nrows = 0;
    for (thm_system *s : sys) {
        nnz += (int64_t)s->K.col.size();
        nrows += s->n;
    }
    const thm_system &s0 = *sys[0];
    int nb = 0;
    while ((int64_t(1) << (nb + 1)) <= nrows) ++nb;
    char key64[128], key32[128];
    std::snprintf(key64, sizeof key64, "gfx950:d%d:p%d:n%d:b%d:fp64", s0.topo.dim, s0.topo.p, nb, ns);
    std::snprintf(key32, sizeof key32, "gfx950:d%d:p%d:n%d:b%d:fp32", s0.topo.dim, s0.topo.p, nb, ns);
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
        const Sched &sc = K.B.spmv_sched(c, st);
        const float ms = time_it([&] {
            launch_spmv<double>(c, mat64.p, K.B.off.p, sc, ns, nullptr, x64.p, r64.p, nullptr, 1.f, st);
        });
        if (ms < best) { best = ms; lpr64 = c; }
    }
    ops32(1.f);
    best = 1e30f;
    for (int c : cand) {
        const Sched &sc = K.B.spmv_sched(c, st);
        const float ms = time_it([&] {
            launch_spmv<float>(c, mat32.p, K.B.off.p, sc, ns, nullptr, x32.p, b32.p, nullptr, 1.f, st);
        });
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
