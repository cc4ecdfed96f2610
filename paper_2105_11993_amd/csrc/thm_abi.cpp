// C ABI of the THM library: assembly (eqs. (2)-(4)), block-preconditioned GMRES
// (eq. (11)), the impedance-transmission domain decomposition (eqs. (5)-(10)) and
// the adjoint gradient.  Exceptions never cross the interface: every entry point
// catches, stores a thread-local message and returns a thm_status.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>

#include "solver.h"

namespace thm {

static thread_local std::string g_last_error;

void fail(thm_status code, const std::string &msg) { throw Error{code, msg}; }

template <class F>
static thm_status guard(F &&f) {
    try {
        f();
        return THM_OK;
    } catch (const Error &e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return THM_ENOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return THM_EINVAL;
    } catch (...) {
        g_last_error = "unknown internal error";
        return THM_EINVAL;
    }
}

// Counting sort (key -> list of values) into CSR arrays.
static void bucket(int64_t nkeys, const std::vector<int64_t> &key, const std::vector<int32_t> &val,
                   std::vector<int32_t> &ptr, std::vector<int32_t> &out) {
    ptr.assign(nkeys + 1, 0);
    for (int64_t k : key) ptr[k + 1]++;
    for (int64_t i = 0; i < nkeys; ++i) ptr[i + 1] += ptr[i];
    out.assign(val.size(), 0);
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (size_t i = 0; i < key.size(); ++i) out[fill[key[i]]++] = val[i];
}

// ---------------------------------------------------------------- DDM data
struct Ddm {
    int nsub = 0;
    int S[3] = {1, 1, 1};
    int64_t nent = 0, ntouch = 0;
    DBuf<int32_t> ent_sys, ent_row, ent_rev, ent_mptr, m_col;
    DBuf<double> m_val;
    DBuf<int32_t> touch_sys, touch_dof, touch_ptr, touch_src;
    DBuf<int32_t> own_sys, own_loc;
    // solve-time state
    std::unique_ptr<Ctx> inner;
    std::vector<std::unique_ptr<Ctx>> singles;
    DBuf<double *> Xb, Bb, Xs, Bs;  // per-subdomain slot pointers (batched / sequential contexts)
    std::unique_ptr<Krylov> outer;
    DBuf<double> G, Gb, tmp, Eg, minus1;
    DBuf<int32_t> one;
    Batch Bg;                       // single-system batch over the global system
    DBuf<MatDesc> gmat;
    DBuf<const uint8_t *> gdir;
    DBuf<double> gres, gr2, gpart, gnorm;
    int inner_iters = 0;
};

}  // namespace thm

using namespace thm;

thm_system::~thm_system() = default;

// ---------------------------------------------------------------- context caches
static std::mutex g_cache_mu;
static std::map<std::vector<thm_system *>, std::unique_ptr<Ctx>> g_ctx_cache;

static void drop_contexts(thm_system *s) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (auto it = g_ctx_cache.begin(); it != g_ctx_cache.end();) {
        if (std::find(it->first.begin(), it->first.end(), s) != it->first.end()) {
            if (it->second && it->second->st) (void)hipStreamSynchronize(it->second->st);
            it = g_ctx_cache.erase(it);
        } else {
            ++it;
        }
    }
    if (s->ddm) {
        s->ddm->inner.reset();
        s->ddm->singles.clear();
    }
}

static Ctx &get_ctx(const std::vector<thm_system *> &sys, int m) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto &slot = g_ctx_cache[sys];
    if (slot && slot->K.m != m) slot.reset();
    if (!slot) {
        auto c = std::make_unique<Ctx>();
        hipStream_t st;
        THM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        try {
            c->build(sys, m, st);
        } catch (...) {
            (void)hipStreamDestroy(st);
            throw;
        }
        slot = std::move(c);
    }
    return *slot;
}

// Order the internal stream after the caller's stream (and vice versa at the end).
static void stream_join(hipStream_t from, hipStream_t to) {
    hipEvent_t e;
    THM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    THM_HIP(hipEventRecord(e, from));
    THM_HIP(hipStreamWaitEvent(to, e, 0));
    THM_HIP(hipEventDestroy(e));
}

// ---------------------------------------------------------------- validation
static void validate(const thm_problem *p) {
    if (!p) fail(THM_EINVAL, "problem is NULL");
    if (p->dim != 2 && p->dim != 3) fail(THM_EUNSUPPORTED, "dim must be 2 or 3");
    if (p->degree < 0) fail(THM_EINVAL, "degree must be >= 0");
    if ((p->dim == 2 && p->degree > 3) || (p->dim == 3 && p->degree > 1))
        fail(THM_EUNSUPPORTED, "supported degrees: 2D p <= 3, 3D p <= 1");
    int64_t nc = 1;
    for (int a = 0; a < p->dim; ++a) {
        if (p->cells[a] < 1) fail(THM_EINVAL, "cells must be >= 1");
        if (!(p->box_hi[a] > p->box_lo[a]) || !std::isfinite(p->box_hi[a]) || !std::isfinite(p->box_lo[a]))
            fail(THM_EINVAL, "box_hi must exceed box_lo");
        nc *= p->cells[a];
        const int sd = p->subdomains[a] < 1 ? 1 : p->subdomains[a];
        if (p->cells[a] % sd) fail(THM_EUNSUPPORTED, "cells must divide evenly into subdomains");
    }
    if (!(p->omega > 0.0) || !std::isfinite(p->omega)) fail(THM_EINVAL, "omega must be > 0");
    if (!(p->kappa > 0.0) || !std::isfinite(p->kappa)) fail(THM_EINVAL, "kappa must be > 0");
    const uint32_t all = (1u << (2 * p->dim)) - 1u;
    if ((p->inc_faces & all) == all) fail(THM_EINVAL, "Gamma^inf is empty: at least one side must be impedance");
    if (p->mu)
        for (int64_t c = 0; c < nc; ++c)
            if (!(p->mu[c] > 0.0) || !std::isfinite(p->mu[c])) fail(THM_EINVAL, "mu must be finite and > 0");
    if (p->eps)
        for (int64_t c = 0; c < nc; ++c)
            if (!(p->eps[c] > 0.0) || !std::isfinite(p->eps[c])) fail(THM_EINVAL, "eps must be finite and > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->inc_dir[a]) || !std::isfinite(p->inc_pol_re[a]) || !std::isfinite(p->inc_pol_im[a]))
            fail(THM_EINVAL, "incident field parameters must be finite");
    if (!std::isfinite(p->transmission[0]) || !std::isfinite(p->transmission[1]))
        fail(THM_EINVAL, "transmission factor must be finite");
}

// ---------------------------------------------------------------- Dirichlet projection (Jacobi-PCG)
static void project_dirichlet(thm_system &S, hipStream_t st) {
    const int64_t n = S.n;
    DBuf<int32_t> zptr(n + 1);
    THM_HIP(hipMemsetAsync(zptr.p, 0, sizeof(int32_t) * (n + 1), st));
    DBuf<int32_t> mrp, mcol, mgp, mgs;
    mrp.upload(S.Minc.rowptr, st);
    mcol.upload(S.Minc.col, st);
    mgp.upload(S.Minc.gptr, st);
    mgs.upload(S.Minc.gsrc, st);
    const int nsi = (int)S.sides_inc.size(), nf = S.nf;
    DBuf<double> mblk((size_t)nsi * nf * nf), mval(std::max<size_t>(S.Minc.col.size(), 1));
    const FeTables *ts[6] = {&S.tside, &S.tside, &S.tside, &S.tside, &S.tside, &S.tside};
    launch_side_mass(S.topo.dim, nsi, S.si_axis.p, S.si_side.p, S.side_fn.p, nf, S.topo.n_loc, ts, S.h.p, mblk.p, st);
    launch_gather((int64_t)S.Minc.col.size(), mgp.p, mgs.p, mblk.p, 1.0, mval.p, st);
    // load s (complex) gathered from per-side loads
    DBuf<double> lblk((size_t)nsi * nf * 2);
    const FeTables *tl[6] = {&S.tload, &S.tload, &S.tload, &S.tload, &S.tload, &S.tload};
    DBuf<double> dirv(3), pre(3), pim(3);
    THM_HIP(hipMemcpyAsync(dirv.p, S.prob.inc_dir, 3 * sizeof(double), hipMemcpyHostToDevice, st));
    THM_HIP(hipMemcpyAsync(pre.p, S.prob.inc_pol_re, 3 * sizeof(double), hipMemcpyHostToDevice, st));
    THM_HIP(hipMemcpyAsync(pim.p, S.prob.inc_pol_im, 3 * sizeof(double), hipMemcpyHostToDevice, st));
    launch_side_load(S.topo.dim, nsi, S.si_cell.p, S.si_axis.p, S.si_side.p, S.side_fn.p, nf, S.topo.n_loc, tl, S.h.p,
                     S.lo.p, S.ncell.p, dirv.p, pre.p, pim.p, S.prob.omega, lblk.p, st);
    std::vector<int64_t> key;
    std::vector<int32_t> val;
    const int nl = S.topo.n_loc;
    for (int si = 0; si < nsi; ++si) {
        const Side &sd = S.sides_inc[si];
        const auto &sf = S.topo.side_fns[2 * sd.axis + sd.side];
        for (int a = 0; a < nf; ++a) {
            key.push_back(S.topo.cell_dofs[(size_t)sd.cell * nl + sf[a]]);
            val.push_back(si * nf + a);
        }
    }
    std::vector<int32_t> lp, ls;
    bucket(n, key, val, lp, ls);
    DBuf<int32_t> lpd, lsd;
    lpd.upload(lp, st);
    lsd.upload(ls, st);
    DBuf<double> s(2 * n), r(2 * n), z(2 * n), p(2 * n), q(2 * n), d(n), sc(8);
    launch_gather_vec(n, lpd.p, lsd.p, lblk.p, s.p, st);
    launch_diag_extract(n, mrp.p, mcol.p, mval.p, d.p, st);
    // operator: the Gamma^inc mass (real) acting on complex vectors
    Batch B1;
    B1.init({n}, 2, st);
    MatDesc md{n, mrp.p, mcol.p, mval.p, zptr.p, zptr.p, mval.p};
    DBuf<MatDesc> mdd;
    mdd.upload(std::vector<MatDesc>{md}, st);
    const Sched &sc8 = B1.spmv_sched(81, st);
    const int64_t m2 = 2 * n;
    THM_HIP(hipMemsetAsync(S.gD.p, 0, sizeof(double) * m2, st));
    THM_HIP(hipMemcpyAsync(r.p, s.p, sizeof(double) * m2, hipMemcpyDeviceToDevice, st));
    launch_diag_solve(n, d.p, r.p, z.p, st);
    THM_HIP(hipMemcpyAsync(p.p, z.p, sizeof(double) * m2, hipMemcpyDeviceToDevice, st));
    launch_dot1(m2, r.p, z.p, sc.p + 0, st);
    launch_dot1(m2, s.p, s.p, sc.p + 5, st);
    double hs[8];
    THM_HIP(hipMemcpyAsync(hs, sc.p, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
    THM_HIP(hipStreamSynchronize(st));
    const double bn = std::sqrt(hs[5]);
    if (bn == 0.0) return;
    for (int it = 0; it < 1000; ++it) {
        launch_spmv<double>(81, mdd.p, B1.off.p, sc8, 1, nullptr, p.p, q.p, nullptr, 0.f, st);
        launch_dot1(m2, p.p, q.p, sc.p + 1, st);
        launch_cg_step(m2, 0, sc.p, S.gD.p, p.p, r.p, q.p, nullptr, nullptr, st);
        launch_dot1(m2, r.p, r.p, sc.p + 4, st);
        THM_HIP(hipMemcpyAsync(hs, sc.p, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
        THM_HIP(hipStreamSynchronize(st));
        if (!(std::sqrt(hs[4]) > 1e-15 * bn)) break;
        launch_diag_solve(n, d.p, r.p, z.p, st);
        launch_dot1(m2, r.p, z.p, sc.p + 2, st);
        THM_HIP(hipMemcpyAsync(sc.p + 3, sc.p + 0, sizeof(double), hipMemcpyDeviceToDevice, st));
        launch_cg_step(m2, 1, sc.p + 2, nullptr, nullptr, nullptr, nullptr, p.p, z.p, st);
        THM_HIP(hipMemcpyAsync(sc.p + 0, sc.p + 2, sizeof(double), hipMemcpyDeviceToDevice, st));
    }
}

// rhs = -S_FD gD on free rows, 0 on Dirichlet rows
static void compute_lift(thm_system &S, hipStream_t st) {
    Batch B1;
    B1.init({S.n}, 2, st);
    MatDesc md{S.n, S.k_rowptr.p, S.k_col.p, S.kraw.p, S.c_rowptr.p, S.c_col.p, S.craw.p};
    DBuf<MatDesc> mdd;
    mdd.upload(std::vector<MatDesc>{md}, st);
    launch_spmv<double>(81, mdd.p, B1.off.p, B1.spmv_sched(81, st), 1, nullptr, S.gD.p, S.rhs.p, nullptr, 1.f, st);
    launch_lift_finish(S.n, S.dir_d.p, S.rhs.p, st);
    THM_HIP(hipStreamSynchronize(st));
}

// K values from the current mu: element kernel, gather, Dirichlet rows/columns, FP32 copy.
static void assemble_K(thm_system &S, hipStream_t st) {
    const Topo &t = S.topo;
    launch_element_matrices(t.dim, t.n_cells, t.n_loc, S.tcell, S.h.p, S.mu_d.p, S.eps_d.n ? S.eps_d.p : nullptr,
                            S.prob.omega, S.kel.p, st);
    // DDM interface sides with S = s 1 carry i k w s M_Sigma: its real part -k w Im(s) M_Sigma
    // belongs to K (added to the element matrices, so the factorisation sees it too)
    const double s_im = S.prob.transmission[1];
    if (S.iface_sides && s_im != 0.0) {
        const double coef = -S.prob.kappa * S.prob.omega * s_im;
        for (int g = 0; g < 2 * t.dim; ++g)
            if ((S.iface_sides >> g) & 1u)
                launch_side_to_elem(S.cside_lo[g], S.cside_hi[g], S.sc_cell.p, S.sc_axis.p, S.sc_side.p, S.side_fn.p,
                                    S.nf, t.n_loc, coef, S.cside.p, S.kel.p, st);
    }
    const int64_t nnz = (int64_t)S.K.col.size();
    launch_gather(nnz, S.k_gptr.p, S.k_gsrc.p, S.kel.p, 1.0, S.kraw.p, st);
    THM_HIP(hipMemcpyAsync(S.kval.p, S.kraw.p, sizeof(double) * nnz, hipMemcpyDeviceToDevice, st));
    launch_dirichletize(S.n, S.k_rowptr.p, S.k_col.p, S.dir_d.p, S.kval.p, 1, st);
    launch_convert(S.kval.p, S.kval32.p, nnz, st);
    launch_sell_fill((int64_t)S.sl_src.n, S.sl_src.p, S.kval.p, S.sl_val.p, S.sl_val32.p, st);
}

static void assemble_system(thm_system &S, const thm_problem &p, uint32_t iface_sides, hipStream_t st) {
    S.prob = p;
    S.prob.mu = nullptr;
    S.prob.eps = nullptr;
    if (S.prob.transmission[0] == 0.0 && S.prob.transmission[1] == 0.0) S.prob.transmission[0] = 1.0;
    S.iface_sides = iface_sides;
    Topo &t = S.topo;
    t.build(p.dim, p.degree, p.cells, p.box_lo, p.box_hi);
    S.n = t.n_dofs;
    const int nl = t.n_loc;
    S.mu_host.assign(t.n_cells, 1.0);
    if (p.mu) std::copy(p.mu, p.mu + t.n_cells, S.mu_host.begin());
    S.eps_host.clear();
    if (p.eps) S.eps_host.assign(p.eps, p.eps + t.n_cells);
    S.sides_c.clear();
    S.sides_inc.clear();
    for (int axis = 0; axis < t.dim; ++axis)
        for (int side = 0; side < 2; ++side) {
            const bool inc = (p.inc_faces >> (2 * axis + side)) & 1u;
            S.cside_lo[2 * axis + side] = (int)S.sides_c.size();
            for (int64_t c = 0; c < t.n_cells; ++c)
                if (t.cell_on_side(c, axis, side)) (inc ? S.sides_inc : S.sides_c).push_back({(int32_t)c, axis, side});
            S.cside_hi[2 * axis + side] = (int)S.sides_c.size();
        }
    S.nf = (int)t.side_fns[0].size();
    S.dir.assign(S.n, 0);
    for (const Side &sd : S.sides_inc)
        for (int u : t.side_fns[2 * sd.axis + sd.side]) S.dir[t.cell_dofs[(size_t)sd.cell * nl + u]] = 1;
    S.n_free = S.n - std::count(S.dir.begin(), S.dir.end(), (uint8_t)1);
    build_csr(t, S.K);
    build_side_csr(t, S.sides_c, S.C);
    build_side_csr(t, S.sides_inc, S.Minc);
    build_layering(t, S.dir, S.L);
    S.Lskel_dof.upload(S.L.skel_dof, st);
    S.Lskel_pos.upload(S.L.skel_pos, st);
    {
        // global DoF -> padded position in the skeleton work vectors (-1: interior)
        std::vector<int32_t> vpos(S.L.dof_pos.size(), -1);
        for (size_t g = 0; g < vpos.size(); ++g)
            if (S.L.dof_pos[g] >= 0) vpos[g] = S.L.skel_pos[S.L.dof_pos[g]];
        S.Ldof_pos.upload(vpos, st);
        // per cell: padded positions of its skeleton (non-interior) local DoFs
        const int ne = t.n_loc - t.n_int;
        std::vector<int32_t> cpos((size_t)t.n_cells * ne);
        for (int64_t c = 0; c < t.n_cells; ++c)
            for (int le = 0; le < ne; ++le) cpos[(size_t)c * ne + le] = vpos[t.cell_dofs[(size_t)c * t.n_loc + le]];
        S.Lcell_pos.upload(cpos, st);
    }
    S.Lcond_ptr.upload(S.L.cond_ptr, st);
    S.Lcond_cell.upload(S.L.cond_cell, st);
    S.Lcond_loc.upload(S.L.cond_loc, st);
    {
        std::vector<int64_t> key((size_t)t.n_cells * nl);
        std::vector<int32_t> val(key.size());
        for (size_t i = 0; i < key.size(); ++i) {
            key[i] = t.cell_dofs[i];
            val[i] = (int32_t)i;
        }
        std::vector<int32_t> dp, ds;
        bucket(S.n, key, val, dp, ds);
        S.d2c_ptr.upload(dp, st);
        S.d2c_src.upload(ds, st);
    }
    // uploads
    S.fns.upload(t.fns, st);
    S.cell_dofs.upload(t.cell_dofs, st);
    S.k_rowptr.upload(S.K.rowptr, st);
    S.k_col.upload(S.K.col, st);
    S.k_gptr.upload(S.K.gptr, st);
    S.k_gsrc.upload(S.K.gsrc, st);
    S.c_rowptr.upload(S.C.rowptr, st);
    S.c_col.upload(S.C.col, st);
    S.c_gptr.upload(S.C.gptr, st);
    S.c_gsrc.upload(S.C.gsrc, st);
    {
        std::vector<int32_t> sf((size_t)2 * t.dim * std::max(S.nf, 1), 0);
        for (int s6 = 0; s6 < 2 * t.dim; ++s6)
            for (int a = 0; a < S.nf; ++a) sf[(size_t)s6 * S.nf + a] = t.side_fns[s6][a];
        S.side_fn.upload(sf, st);
        std::vector<int32_t> a1, s1, c1, a2, s2, c2;
        for (const Side &sd : S.sides_c) { a1.push_back(sd.axis); s1.push_back(sd.side); c1.push_back(sd.cell); }
        for (const Side &sd : S.sides_inc) { a2.push_back(sd.axis); s2.push_back(sd.side); c2.push_back(sd.cell); }
        S.sc_axis.upload(a1, st);
        S.sc_side.upload(s1, st);
        S.sc_cell.upload(c1, st);
        S.si_axis.upload(a2, st);
        S.si_side.upload(s2, st);
        S.si_cell.upload(c2, st);
    }
    S.h.upload(std::vector<double>(t.h, t.h + 3), st);
    S.lo.upload(std::vector<double>(t.lo, t.lo + 3), st);
    S.ncell.upload(std::vector<int32_t>(t.n, t.n + 3), st);
    S.mu_d.upload(S.mu_host, st);
    if (!S.eps_host.empty()) S.eps_d.upload(S.eps_host, st);
    else S.eps_d.release();
    S.dir_d.upload(S.dir, st);
    // reference tables: cell Gauss q = p+2, side Gauss q = p+2, incident load 10 points per direction
    fe_tables_cell(t.dim, t.p, t.p + 2, S.fns.p, nl, S.tcell, st);
    fe_tables_side(t.dim, t.p, t.p + 2, 0, 0, S.fns.p, nl, S.tside, st);
    fe_tables_side(t.dim, t.p, 10, 0, 0, S.fns.p, nl, S.tload, st);
    // tangential trace masses of the sides carrying C
    const int nsc = (int)S.sides_c.size();
    S.cside.alloc((size_t)std::max(nsc, 1) * S.nf * S.nf);
    {
        const FeTables *ts[6] = {&S.tside, &S.tside, &S.tside, &S.tside, &S.tside, &S.tside};
        launch_side_mass(t.dim, nsc, S.sc_axis.p, S.sc_side.p, S.side_fn.p, S.nf, nl, ts, S.h.p, S.cside.p, st);
    }
    // K
    const int64_t nnz = (int64_t)S.K.col.size();
    S.kel.alloc((size_t)t.n_cells * nl * nl);
    S.kraw.alloc(nnz);
    S.kval.alloc(nnz);
    S.kval32.alloc(nnz);
    {
        std::vector<int32_t> ptr, scol, src, row;
        sell_build(S.n, S.K.rowptr, S.K.col, ptr, scol, src, row);
        S.sl_row.upload(row, st);
        S.sl_ptr.upload(ptr, st);
        S.sl_col.upload(scol, st);
        S.sl_src.upload(src, st);
        S.sl_val.alloc(std::max<size_t>(src.size(), 1));
        S.sl_val32.alloc(std::max<size_t>(src.size(), 1));
    }
    assemble_K(S, st);
    // C = k w (M_inf + Re(s) M_Sigma)
    const int64_t nnzc = (int64_t)S.C.col.size();
    S.craw.alloc(std::max<int64_t>(nnzc, 1));
    S.cval.alloc(std::max<int64_t>(nnzc, 1));
    S.cval32.alloc(std::max<int64_t>(nnzc, 1));
    if (iface_sides && S.prob.transmission[0] != 1.0) {
        DBuf<double> cblk((size_t)std::max(nsc, 1) * S.nf * S.nf);
        launch_side_scale(nsc, S.sc_axis.p, S.sc_side.p, iface_sides, S.nf, S.prob.transmission[0], S.cside.p, cblk.p,
                          st);
        launch_gather(nnzc, S.c_gptr.p, S.c_gsrc.p, cblk.p, p.kappa * p.omega, S.craw.p, st);
        THM_HIP(hipStreamSynchronize(st));
    } else {
        launch_gather(nnzc, S.c_gptr.p, S.c_gsrc.p, S.cside.p, p.kappa * p.omega, S.craw.p, st);
    }
    THM_HIP(hipMemcpyAsync(S.cval.p, S.craw.p, sizeof(double) * nnzc, hipMemcpyDeviceToDevice, st));
    launch_dirichletize(S.n, S.c_rowptr.p, S.c_col.p, S.dir_d.p, S.cval.p, 0, st);
    launch_convert(S.cval.p, S.cval32.p, nnzc, st);
    // Dirichlet data and lifted right-hand side
    S.gD.alloc(2 * S.n);
    S.rhs.alloc(2 * S.n);
    THM_HIP(hipMemsetAsync(S.gD.p, 0, sizeof(double) * 2 * S.n, st));
    if (!S.sides_inc.empty()) project_dirichlet(S, st);
    compute_lift(S, st);
}

// ---------------------------------------------------------------- DDM construction
static void build_ddm(thm_system &G, hipStream_t st) {
    const thm_problem &p = G.prob;
    if (std::getenv("THM_PROGRESS")) std::fprintf(stderr, "[thm] building subdomain systems\n");
    const int d = p.dim;
    auto D = std::make_unique<Ddm>();
    int S[3] = {1, 1, 1}, nloc[3] = {1, 1, 1};
    for (int a = 0; a < d; ++a) {
        S[a] = std::max(1, p.subdomains[a]);
        nloc[a] = p.cells[a] / S[a];
    }
    D->nsub = S[0] * S[1] * S[2];
    std::copy(S, S + 3, D->S);
    // global Dirichlet values (host copy)
    std::vector<double> gD(2 * G.n);
    THM_HIP(hipMemcpyAsync(gD.data(), G.gD.p, sizeof(double) * 2 * G.n, hipMemcpyDeviceToHost, st));
    THM_HIP(hipStreamSynchronize(st));
    const Topo &gt = G.topo;
    std::vector<std::vector<int32_t>> l2g(D->nsub);
    std::vector<std::vector<int32_t>> g2l(D->nsub);
    for (int s = 0; s < D->nsub; ++s) {
        const int pos[3] = {s % S[0], (s / S[0]) % S[1], s / (S[0] * S[1])};
        thm_problem lp = p;
        uint32_t inc = 0, iface = 0;
        for (int a = 0; a < 3; ++a) {
            lp.cells[a] = a < d ? nloc[a] : 1;
            if (a < d) {
                lp.box_lo[a] = gt.lo[a] + pos[a] * nloc[a] * gt.h[a];
                lp.box_hi[a] = lp.box_lo[a] + nloc[a] * gt.h[a];
            }
            lp.subdomains[a] = 1;
        }
        for (int a = 0; a < d; ++a) {
            if (pos[a] == 0) inc |= p.inc_faces & (1u << (2 * a));
            else iface |= 1u << (2 * a);
            if (pos[a] == S[a] - 1) inc |= p.inc_faces & (1u << (2 * a + 1));
            else iface |= 1u << (2 * a + 1);
        }
        lp.inc_faces = inc;
        std::vector<double> mu_l((size_t)nloc[0] * nloc[1] * nloc[2]), eps_l;
        if (!G.eps_host.empty()) eps_l.resize(mu_l.size());
        for (size_t c = 0; c < mu_l.size(); ++c) {
            const int i = (int)(c % nloc[0]), j = (int)((c / nloc[0]) % nloc[1]), k = (int)(c / ((size_t)nloc[0] * nloc[1]));
            const int64_t gc = ((int64_t)(k + pos[2] * nloc[2]) * p.cells[1] + (j + pos[1] * nloc[1])) * p.cells[0] +
                               (i + pos[0] * nloc[0]);
            mu_l[c] = G.mu_host[gc];
            if (!eps_l.empty()) eps_l[c] = G.eps_host[gc];
        }
        lp.mu = mu_l.data();
        lp.eps = eps_l.empty() ? nullptr : eps_l.data();
        auto sub = std::make_unique<thm_system>();
        assemble_system(*sub, lp, iface, st);
        const Topo &lt = sub->topo;
        l2g[s].assign(sub->n, -1);
        for (int64_t c = 0; c < lt.n_cells; ++c) {
            int ijk[3];
            lt.cell_ijk(c, ijk);
            const int64_t gc = ((int64_t)(ijk[2] + pos[2] * nloc[2]) * gt.n[1] + (ijk[1] + pos[1] * nloc[1])) * gt.n[0] +
                               (ijk[0] + pos[0] * nloc[0]);
            for (int u = 0; u < lt.n_loc; ++u)
                l2g[s][lt.cell_dofs[(size_t)c * lt.n_loc + u]] = gt.cell_dofs[(size_t)gc * gt.n_loc + u];
        }
        g2l[s].assign(G.n, -1);
        for (int64_t l = 0; l < sub->n; ++l) g2l[s][l2g[s][l]] = (int32_t)l;
        // Dirichlet values from the global projection, then the lift again
        std::vector<double> lg(2 * sub->n, 0.0);
        for (int64_t l = 0; l < sub->n; ++l)
            if (sub->dir[l]) {
                lg[2 * l] = gD[2 * (size_t)l2g[s][l]];
                lg[2 * l + 1] = gD[2 * (size_t)l2g[s][l] + 1];
            }
        THM_HIP(hipMemcpyAsync(sub->gD.p, lg.data(), sizeof(double) * lg.size(), hipMemcpyHostToDevice, st));
        compute_lift(*sub, st);
        G.subs.push_back(std::move(sub));
    }
    // interfaces: entries [a->b block][b->a block] per face-adjacent pair
    struct Ent { int sys, row, rev; std::vector<int32_t> cols; std::vector<std::pair<int, int>> src; };
    std::vector<int32_t> e_sys, e_row, e_rev, m_ptr(1, 0), m_col, m_gptr(1, 0), m_gsrc;
    std::vector<double> dummy;
    std::vector<std::pair<int, int64_t>> blk_owner;  // (subdomain, side) per side-block batch
    // side-mass blocks of interface sides, computed per subdomain on its tables
    std::vector<double> mval_all;
    DBuf<double> mval_dev;
    int64_t mval_total = 0;
    struct Pending { int sub; int axis, side; std::vector<Side> sides; int64_t base; };
    std::vector<Pending> pend;
    const int nfl = G.subs[0]->nf;
    auto side_cells = [&](int s, int axis, int side) {
        std::vector<Side> out;
        const Topo &lt = G.subs[s]->topo;
        for (int64_t c = 0; c < lt.n_cells; ++c)
            if (lt.cell_on_side(c, axis, side)) out.push_back({(int32_t)c, axis, side});
        return out;
    };
    std::vector<std::pair<int64_t, int32_t>> touch;  // ((recv sys << 32) | dof, entry)
    for (int s = 0; s < D->nsub; ++s) {
        const int pos[3] = {s % S[0], (s / S[0]) % S[1], s / (S[0] * S[1])};
        for (int a = 0; a < d; ++a) {
            if (pos[a] + 1 >= S[a]) continue;
            int pt[3] = {pos[0], pos[1], pos[2]};
            pt[a] += 1;
            const int t = (pt[2] * S[1] + pt[1]) * S[0] + pt[0];
            const thm_system &A = *G.subs[s], &Bs = *G.subs[t];
            std::set<int32_t> gset;
            for (const Side &sd : side_cells(s, a, 1))
                for (int u : A.topo.side_fns[2 * a + 1]) {
                    const int32_t g = l2g[s][A.topo.cell_dofs[(size_t)sd.cell * A.topo.n_loc + u]];
                    if (!G.dir[g]) gset.insert(g);
                }
            std::vector<int32_t> gl(gset.begin(), gset.end());
            const int mcount = (int)gl.size();
            const int64_t e0 = (int64_t)e_sys.size();
            for (int dirn = 0; dirn < 2; ++dirn) {
                const int snd = dirn == 0 ? s : t, rcv = dirn == 0 ? t : s;
                const int sside = dirn == 0 ? 1 : 0;
                const thm_system &Sx = dirn == 0 ? A : Bs;
                std::vector<Side> sides = side_cells(snd, a, sside);
                // rows: the interface DoFs in sender numbering; columns/gather from side blocks
                std::vector<std::vector<std::pair<int32_t, int32_t>>> rowent(mcount);
                std::map<int32_t, int> rowidx;
                for (int i = 0; i < mcount; ++i) rowidx[g2l[snd][gl[i]]] = i;
                const auto &sf = Sx.topo.side_fns[2 * a + sside];
                for (size_t si = 0; si < sides.size(); ++si) {
                    const int32_t *cd = &Sx.topo.cell_dofs[(size_t)sides[si].cell * Sx.topo.n_loc];
                    for (int aa = 0; aa < nfl; ++aa) {
                        auto it = rowidx.find(cd[sf[aa]]);
                        if (it == rowidx.end()) continue;
                        for (int bb = 0; bb < nfl; ++bb)
                            rowent[it->second].push_back(
                                {cd[sf[bb]], (int32_t)(mval_total + ((int64_t)si * nfl + aa) * nfl + bb)});
                    }
                }
                pend.push_back({snd, a, sside, sides, mval_total});
                mval_total += (int64_t)sides.size() * nfl * nfl;
                for (int i = 0; i < mcount; ++i) {
                    auto &re = rowent[i];
                    std::sort(re.begin(), re.end());
                    size_t q = 0;
                    while (q < re.size()) {
                        const int32_t col = re[q].first;
                        m_col.push_back(col);
                        while (q < re.size() && re[q].first == col) m_gsrc.push_back(re[q++].second);
                        m_gptr.push_back((int32_t)m_gsrc.size());
                    }
                    m_ptr.push_back((int32_t)m_col.size());
                    e_sys.push_back(snd);
                    e_row.push_back(g2l[snd][gl[i]]);
                    e_rev.push_back((int32_t)(e0 + (dirn == 0 ? mcount + i : i)));
                    const int64_t e = (int64_t)e_sys.size() - 1;
                    touch.push_back({((int64_t)rcv << 32) | (int64_t)g2l[rcv][gl[i]], (int32_t)e});
                }
            }
        }
    }
    D->nent = (int64_t)e_sys.size();
    D->ent_sys.upload(e_sys, st);
    D->ent_row.upload(e_row, st);
    D->ent_rev.upload(e_rev, st);
    D->ent_mptr.upload(m_ptr, st);
    D->m_col.upload(m_col, st);
    // side blocks, then gather into m_val
    DBuf<double> blocks(std::max<int64_t>(mval_total, 1));
    for (const Pending &pd : pend) {
        const thm_system &Sx = *G.subs[pd.sub];
        std::vector<int32_t> ax(pd.sides.size(), pd.axis), sd(pd.sides.size(), pd.side);
        DBuf<int32_t> axd, sdd;
        axd.upload(ax, st);
        sdd.upload(sd, st);
        const FeTables *ts[6] = {&Sx.tside, &Sx.tside, &Sx.tside, &Sx.tside, &Sx.tside, &Sx.tside};
        launch_side_mass(d, (int)pd.sides.size(), axd.p, sdd.p, Sx.side_fn.p, nfl, Sx.topo.n_loc, ts, Sx.h.p,
                         blocks.p + pd.base, st);
        THM_HIP(hipStreamSynchronize(st));
    }
    {
        DBuf<int32_t> gp, gs;
        gp.upload(m_gptr, st);
        gs.upload(m_gsrc, st);
        D->m_val.alloc(std::max<size_t>(m_col.size(), 1));
        launch_gather((int64_t)m_col.size(), gp.p, gs.p, blocks.p, 1.0, D->m_val.p, st);
        THM_HIP(hipStreamSynchronize(st));
    }
    // incoming data scatter map
    std::sort(touch.begin(), touch.end());
    std::vector<int32_t> ts_, td_, tp_(1, 0), tsrc;
    for (size_t q = 0; q < touch.size();) {
        const int64_t k = touch[q].first;
        ts_.push_back((int32_t)(k >> 32));
        td_.push_back((int32_t)(k & 0xffffffff));
        while (q < touch.size() && touch[q].first == k) tsrc.push_back(touch[q++].second);
        tp_.push_back((int32_t)tsrc.size());
    }
    D->ntouch = (int64_t)ts_.size();
    D->touch_sys.upload(ts_, st);
    D->touch_dof.upload(td_, st);
    D->touch_ptr.upload(tp_, st);
    D->touch_src.upload(tsrc, st);
    // glue owner map (lowest subdomain id)
    std::vector<int32_t> os(G.n, -1), ol(G.n, -1);
    for (int s = 0; s < D->nsub; ++s)
        for (int64_t l = 0; l < (int64_t)l2g[s].size(); ++l) {
            const int32_t g = l2g[s][l];
            if (os[g] < 0) { os[g] = s; ol[g] = (int32_t)l; }
        }
    D->own_sys.upload(os, st);
    D->own_loc.upload(ol, st);
    // global residual helpers
    D->Bg.init({G.n}, 2, st);
    D->gmat.upload(std::vector<MatDesc>{{G.n, G.k_rowptr.p, G.k_col.p, G.kval.p, G.c_rowptr.p, G.c_col.p, G.cval.p}}, st);
    D->gdir.upload(std::vector<const uint8_t *>{G.dir_d.p}, st);
    D->gres.alloc(2 * G.n);
    D->gr2.alloc(2 * G.n);
    D->gpart.alloc((size_t)std::max(1, D->Bg.vs.nblocks) * NPW * D->Bg.maxcols);
    D->gnorm.alloc(2);
    D->Eg.alloc(2 * G.n);
    D->minus1.upload(std::vector<double>{-1.0}, st);
    D->one.upload(std::vector<int32_t>{1}, st);
    D->Bg.spmv_sched(81, st);
    THM_HIP(hipStreamSynchronize(st));
    G.ddm = std::move(D);
}

// ---------------------------------------------------------------- DDM solve
namespace {

struct DdmRun {
    thm_system &G;
    Ddm &D;
    thm_solve_opts inner_o;
    bool batched;
    hipStream_t st;
    int sweeps_inner_iters = 0;
    int fallbacks = 0;  // subdomain solves finished in FP64 (THM_FP32_IR)
    int gmres_ir = 0;   // subdomain solves finished by GMRES-IR (THM_FP32_IR)

    // E_s for all subdomains given interface data Gv (nullable = 0) and the incident flag.
    void inner_solve(const double *Gv, bool incident) {
        THM_HIP(hipStreamSynchronize(st));
        const int ns = D.nsub;
        std::vector<int> it, rf;
        std::vector<double> rs;
        int maxit = 0;
        if (batched) {
            Ctx &c = *D.inner;
            if (incident) {
                for (int s = 0; s < ns; ++s)
                    THM_HIP(hipMemcpyAsync(c.b64.p + c.K.B.h_off[s], G.subs[s]->rhs.p,
                                           sizeof(double) * 2 * G.subs[s]->n, hipMemcpyDeviceToDevice, c.st));
            } else {
                THM_HIP(hipMemsetAsync(c.b64.p, 0, sizeof(double) * c.b64.n, c.st));  // every slot at once
            }
            if (Gv) launch_ddm_rhs(D.ntouch, D.touch_sys.p, D.touch_dof.p, D.touch_ptr.p, D.touch_src.p, D.Bb.p, Gv, c.st);
            THM_HIP(hipMemsetAsync(c.x64.p, 0, sizeof(double) * c.x64.n, c.st));
            c.solve(inner_o, 1.f, nullptr, it, rf, rs);
            for (int v : it) maxit = std::max(maxit, v);
            for (int f : c.last_fb) fallbacks += f;
            for (int f : c.last_ir) gmres_ir += f;
            if (incident)
                for (int s = 0; s < ns; ++s)
                    launch_expand_dirichlet(G.subs[s]->n, G.subs[s]->dir_d.p, G.subs[s]->gD.p,
                                            c.x64.p + c.K.B.h_off[s], c.st);
        } else {
            for (int s = 0; s < ns; ++s) {
                Ctx &c = *D.singles[s];
                if (incident)
                    THM_HIP(hipMemcpyAsync(c.b64.p, G.subs[s]->rhs.p, sizeof(double) * 2 * G.subs[s]->n,
                                           hipMemcpyDeviceToDevice, c.st));
                else THM_HIP(hipMemsetAsync(c.b64.p, 0, sizeof(double) * 2 * G.subs[s]->n, c.st));
                THM_HIP(hipStreamSynchronize(c.st));
            }
            if (Gv) {
                THM_HIP(hipStreamSynchronize(st));
                launch_ddm_rhs(D.ntouch, D.touch_sys.p, D.touch_dof.p, D.touch_ptr.p, D.touch_src.p, D.Bs.p, Gv, st);
                THM_HIP(hipStreamSynchronize(st));
            }
            for (int s = 0; s < ns; ++s) {
                Ctx &c = *D.singles[s];
                THM_HIP(hipMemsetAsync(c.x64.p, 0, sizeof(double) * c.x64.n, c.st));
                c.solve(inner_o, 1.f, nullptr, it, rf, rs);
                maxit = std::max(maxit, it[0]);
                fallbacks += c.last_fb[0];
                gmres_ir += c.last_ir[0];
                if (incident)
                    launch_expand_dirichlet(G.subs[s]->n, G.subs[s]->dir_d.p, G.subs[s]->gD.p, c.x64.p, c.st);
                THM_HIP(hipStreamSynchronize(c.st));
            }
        }
        sweeps_inner_iters += maxit;
    }
    hipStream_t inner_stream() const { return batched ? D.inner->st : st; }
    const double *const *X() const { return batched ? D.Xb.p : D.Xs.p; }
    void sync_inner() {
        if (batched) THM_HIP(hipStreamSynchronize(D.inner->st));
    }
    // out = mode 0: update(Gv, E); mode 1: Gv - update(Gv, E)
    void update(const double *Gv, int mode, double *out) {
        sync_inner();
        launch_ddm_update(D.nent, D.ent_sys.p, D.ent_row.p, D.ent_rev.p, D.ent_mptr.p, D.m_col.p, D.m_val.p, X(), Gv,
                          G.prob.kappa * G.prob.omega, G.prob.transmission[0], G.prob.transmission[1], mode, out,
                          st);
    }
    double global_residual(double *Eout) {
        sync_inner();
        launch_ddm_glue(G.n, D.own_sys.p, D.own_loc.p, X(), D.Eg.p, st);
        if (Eout) THM_HIP(hipMemcpyAsync(Eout, D.Eg.p, sizeof(double) * 2 * G.n, hipMemcpyDeviceToDevice, st));
        THM_HIP(hipMemcpyAsync(D.gres.p, D.Eg.p, sizeof(double) * 2 * G.n, hipMemcpyDeviceToDevice, st));
        launch_zero_flagged<double>(D.Bg, D.gdir.p, D.gres.p, st);
        const Sched &sc = D.Bg.spmv_sched(81, st);
        launch_spmv<double>(81, D.gmat.p, D.Bg.off.p, sc, 1, nullptr, D.gres.p, D.gr2.p, G.rhs.p, 1.f, st);
        launch_norm2<double>(D.Bg, nullptr, D.gr2.p, D.gpart.p, st);
        launch_norm_finish(D.Bg, D.gpart.p, nullptr, D.gnorm.p, nullptr, 0.0, nullptr, nullptr, st);
        launch_norm2<double>(D.Bg, nullptr, G.rhs.p, D.gpart.p, st);
        launch_norm_finish(D.Bg, D.gpart.p, nullptr, D.gnorm.p + 1, nullptr, 0.0, nullptr, nullptr, st);
        double h[2];
        THM_HIP(hipMemcpyAsync(h, D.gnorm.p, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        THM_HIP(hipStreamSynchronize(st));
        return h[1] > 0.0 ? h[0] / h[1] : 0.0;
    }
};

}  // namespace

// Smallest singular value of the k x k upper triangular complex matrix R (column-major,
// interleaved (re, im), leading dimension ld complex entries), by inverse iteration on R^H R:
// x <- R^{-1} R^{-H} x, normalised; ||R^{-1} R^{-H} x|| -> 1 / sigma_min^2.
static double sigma_min_upper(const std::vector<double> &R, int k, int ld) {
    if (k <= 0) return 1.0;
    auto re = [&](int i, int j) { return R[2 * ((int64_t)j * ld + i)]; };
    auto im = [&](int i, int j) { return R[2 * ((int64_t)j * ld + i) + 1]; };
    std::vector<double> xr(k, 1.0 / std::sqrt((double)k)), xi(k, 0.0), yr(k), yi(k);
    double lam = 0.0;
    for (int it = 0; it < 12; ++it) {
        // R^H y = x (forward substitution): y_i = (x_i - sum_{l<i} conj(R_li) y_l) / conj(R_ii)
        for (int i = 0; i < k; ++i) {
            double ar = xr[i], ai = xi[i];
            for (int l = 0; l < i; ++l) {
                const double rr = re(l, i), ri = -im(l, i);
                ar -= rr * yr[l] - ri * yi[l];
                ai -= rr * yi[l] + ri * yr[l];
            }
            const double dr = re(i, i), di = -im(i, i), den = dr * dr + di * di;
            if (!(den > 0.0)) return 0.0;
            yr[i] = (ar * dr + ai * di) / den;
            yi[i] = (ai * dr - ar * di) / den;
        }
        // R z = y (back substitution), z overwrites x
        for (int i = k - 1; i >= 0; --i) {
            double ar = yr[i], ai = yi[i];
            for (int l = i + 1; l < k; ++l) {
                const double rr = re(i, l), ri = im(i, l);
                ar -= rr * xr[l] - ri * xi[l];
                ai -= rr * xi[l] + ri * xr[l];
            }
            const double dr = re(i, i), di = im(i, i), den = dr * dr + di * di;
            xr[i] = (ar * dr + ai * di) / den;
            xi[i] = (ai * dr - ar * di) / den;
        }
        double nz = 0.0;
        for (int i = 0; i < k; ++i) nz += xr[i] * xr[i] + xi[i] * xi[i];
        nz = std::sqrt(nz);
        if (!(nz > 0.0) || !std::isfinite(nz)) return 0.0;
        lam = nz;
        for (int i = 0; i < k; ++i) {
            xr[i] /= nz;
            xi[i] /= nz;
        }
    }
    return 1.0 / std::sqrt(lam);
}

static void ddm_prepare(thm_system &G, const thm_solve_opts &o, bool batched, hipStream_t st) {
    Ddm &D = *G.ddm;
    if (std::getenv("THM_PROGRESS"))
        std::fprintf(stderr, "[thm] ddm prepare (%s, %d subdomains)\n", batched ? "batched" : "sequential", D.nsub);
    std::vector<thm_system *> subs;
    for (auto &s : G.subs) subs.push_back(s.get());
    if (batched) {
        if (!D.inner || D.inner->K.m != o.restart) {
            D.inner.reset();
            auto c = std::make_unique<Ctx>();
            hipStream_t cs;
            THM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            c->build(subs, o.restart, cs);
            D.inner = std::move(c);
            std::vector<double *> xb, bb;
            for (int s = 0; s < D.nsub; ++s) {
                xb.push_back(D.inner->x64.p + D.inner->K.B.h_off[s]);
                bb.push_back(D.inner->b64.p + D.inner->K.B.h_off[s]);
            }
            D.Xb.upload(xb, st);
            D.Bb.upload(bb, st);
        }
    } else if (D.singles.empty() || D.singles[0]->K.m != o.restart) {
        D.singles.clear();
        setup_precond(subs, st, o.batched != 0);
        std::vector<double *> xs, bs;
        for (int s = 0; s < D.nsub; ++s) {
            auto c = std::make_unique<Ctx>();
            hipStream_t cs;
            THM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            c->build({subs[s]}, o.restart, cs);
            xs.push_back(c->x64.p);
            bs.push_back(c->b64.p);
            D.singles.push_back(std::move(c));
        }
        D.Xs.upload(xs, st);
        D.Bs.upload(bs, st);
    }
    if (!D.outer || D.outer->m != o.outer_restart) {
        D.outer = std::make_unique<Krylov>();
        D.outer->init({D.nent}, o.outer_restart, st);
        D.G.alloc(2 * std::max<int64_t>(D.nent, 1));
        D.Gb.alloc(2 * std::max<int64_t>(D.nent, 1));
        D.tmp.alloc(2 * std::max<int64_t>(D.nent, 1));
    }
    THM_HIP(hipStreamSynchronize(st));
}

static void ddm_solve_impl(thm_system &G, const thm_solve_opts &o, double *E, thm_stats &stt, hipStream_t st) {
    const bool batched = o.batched != 0;
    const double t0 = now_ms();
    ddm_prepare(G, o, batched, st);
    Ddm &D = *G.ddm;
    double setup = 0.0;
    for (auto &s : G.subs) setup = std::max(setup, s->fac ? s->fac->setup_ms : 0.0);
    const double t1 = now_ms();
    thm_solve_opts io = o;
    io.rtol = o.inner_rtol;
    DdmRun run{G, D, io, batched, st};
    int outer = 0;
    double res = 1.0;
    const int64_t m2 = 2 * D.nent;
    if (o.ddm_outer == THM_DDM_JACOBI) {
        THM_HIP(hipMemsetAsync(D.G.p, 0, sizeof(double) * m2, st));
        for (int k = 0; k < o.max_outer; ++k) {
            run.inner_solve(k == 0 ? nullptr : D.G.p, true);
            ++outer;
            if (o.rtol > 0.0) {
                res = run.global_residual(E);
                if (res <= o.rtol) break;
            }
            run.update(D.G.p, 0, D.Gb.p);
            THM_HIP(hipMemcpyAsync(D.G.p, D.Gb.p, sizeof(double) * m2, hipMemcpyDeviceToDevice, st));
        }
        if (!(o.rtol > 0.0)) res = run.global_residual(E);
    } else if (D.nent == 0) {
        run.inner_solve(nullptr, true);
        res = run.global_residual(E);
    } else {
        // b = A(0): incident data with G = 0
        run.inner_solve(nullptr, true);
        THM_HIP(hipMemsetAsync(D.tmp.p, 0, sizeof(double) * m2, st));
        run.update(D.tmp.p, 0, D.Gb.p);
        THM_HIP(hipMemsetAsync(D.G.p, 0, sizeof(double) * m2, st));
        KOps<double> ops;
        const bool progress = std::getenv("THM_PROGRESS") != nullptr;
        int napply = 0;
        GmresParams gp;
        // inexact Krylov relaxation (Simoncini & Szyld, SIAM J. Sci. Comput. 25 (2003)): the
        // operator applied at Arnoldi step k may carry an error up to l * eps / ||r_{k-1}|| with
        // eps the target residual and l the smallest singular value of the outer Hessenberg
        // matrix (their bound also divides by the step count; that worst-case factor is not
        // used).  Relative form: subdomain tolerance max(inner_rtol, min(1e-2, s * rtol / r))
        // with r the outer relative residual estimate after the previous step and s the
        // smallest singular value of the triangular factor R of the current cycle's Hessenberg
        // matrix (the same as the Hessenberg's: the Givens rotations are unitary), kept as the
        // minimum over the run.  1e-2 caps it where FP32 inner solves stop gaining.
        const int ldr = D.outer->m + 1;
        std::vector<double> Rh((size_t)2 * ldr * D.outer->m, 0.0);
        double smin = 1.0;
        int rcols = 0;  // columns of the current cycle's R held in Rh
        ops.apply = [&](const double *x, double *y, const double *b, const int32_t *) {
            THM_HIP(hipStreamSynchronize(st));
            ++napply;
            if (progress && napply % 10 == 0)
                std::fprintf(stderr, "[thm] ddm outer apply %d, inner iterations so far %d, %.1f ms\n", napply,
                             run.sweeps_inner_iters, now_ms() - t1);
            run.inner_o.rtol = o.inner_rtol;
            if (o.relax_inner && !b) {
                // explicit residuals b - A x at restarts stay tight
                int32_t j = 0;
                double r = 1.0;
                THM_HIP(hipMemcpy(&j, D.outer->jcnt.p, sizeof(int32_t), hipMemcpyDeviceToHost));
                if (j > 0) {
                    THM_HIP(hipMemcpy(&r, D.outer->est.p, sizeof(double), hipMemcpyDeviceToHost));
                    if (!(r > 0.0) || !(r < 1.0)) r = 1.0;
                    if (j < rcols) rcols = 0;  // a new cycle
                    THM_HIP(hipMemcpy(Rh.data() + (size_t)2 * ldr * rcols, D.outer->H.p + (size_t)2 * ldr * rcols,
                                      sizeof(double) * 2 * ldr * (j - rcols), hipMemcpyDeviceToHost));
                    rcols = j;
                    smin = std::min(smin, sigma_min_upper(Rh, j, ldr));
                }
                run.inner_o.rtol = std::max(o.inner_rtol, std::min(1e-2, smin * gp.rtol / r));
                if (progress && napply % 10 == 0)
                    std::fprintf(stderr, "[thm]   relaxation: outer estimate %.2e, sigma_min %.2e, inner rtol %.2e\n",
                                 r, smin, run.inner_o.rtol);
            }
            run.inner_solve(x, false);
            run.update(x, 1, b ? D.tmp.p : y);
            if (b) {
                THM_HIP(hipMemcpyAsync(y, b, sizeof(double) * m2, hipMemcpyDeviceToDevice, st));
                launch_axpy<double, double>(D.outer->B, nullptr, D.minus1.p, D.tmp.p, y, st);
            }
            THM_HIP(hipStreamSynchronize(st));
        };
        ops.prec = [&](const double *x, double *y, const int32_t *) {
            THM_HIP(hipMemcpyAsync(y, x, sizeof(double) * m2, hipMemcpyDeviceToDevice, st));
        };
        ops.graphable = false;
        gp.rtol = o.rtol;
        gp.orth = o.orth;
        gp.use_graph = false;
        gp.cplx = o.krylov == THM_KRYLOV_COMPLEX ? 1 : 0;
        int budget = o.max_outer;
        for (int attempt = 0; attempt < 4 && budget > 0; ++attempt) {
            gp.max_iter = budget;
            gmres_run<double>(*D.outer, ops, D.Gb.p, D.G.p, D.one.p, gp, st);
            int32_t used = 0;
            THM_HIP(hipMemcpyAsync(&used, D.outer->iters.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            THM_HIP(hipStreamSynchronize(st));
            outer += used;
            budget -= used;
            run.inner_o.rtol = o.inner_rtol;  // the field itself from tight subdomain solves
            run.inner_solve(D.G.p, true);
            res = run.global_residual(E);
            if (res <= o.rtol) break;
            gp.rtol *= 0.1;
        }
    }
    THM_HIP(hipStreamSynchronize(st));
    stt.status = res <= o.rtol || !(o.rtol > 0.0) ? THM_OK : THM_NOT_CONVERGED;
    stt.iters = run.sweeps_inner_iters;
    stt.outer_iters = outer;
    stt.refinements = 0;
    stt.fp64_fallback = run.fallbacks;
    stt.gmres_ir = run.gmres_ir;
    stt.precond_extra_bytes = 0;
    if (o.precond == THM_PREC_FULL) {
        if (batched) stt.precond_extra_bytes = D.inner ? D.inner->full.bytes : 0;
        else
            for (auto &c : D.singles) stt.precond_extra_bytes += c->full.bytes;
    }
    stt.rel_residual = res;
    stt.setup_ms = setup + (t1 - t0);
    stt.solve_ms = now_ms() - t1;
}

// ---------------------------------------------------------------- C ABI
extern "C" {

void thm_default_opts(thm_solve_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->restart = 50;
    o->max_iter = 5000;
    o->rtol = 1e-8;
    o->precision = THM_FP64;
    o->orth = THM_ORTH_CGS;
    o->transpose = 0;
    o->ddm_outer = THM_DDM_GMRES;
    o->inner_rtol = 1e-10;
    o->max_outer = 500;
    o->outer_restart = 200;
    o->batched = 1;
    o->use_graph = 1;
    o->ir_inner_rtol = 1e-6;
    o->max_refine = 30;
    o->krylov = THM_KRYLOV_COMPLEX;
    o->precond = THM_PREC_BLOCK;
    o->ir_mode = THM_IR_CLASSIC;
}

const char *thm_last_error(void) { return g_last_error.c_str(); }

static void check_opts(const thm_solve_opts *o) {
    if (!o) fail(THM_EINVAL, "opts is NULL");
    if (o->restart < 1 || o->restart > 1000) fail(THM_EINVAL, "restart must be in [1, 1000]");
    if (o->max_iter < 0) fail(THM_EINVAL, "max_iter must be >= 0");
    if (!(o->rtol >= 0.0)) fail(THM_EINVAL, "rtol must be >= 0");
    if (o->precision != THM_FP64 && o->precision != THM_FP32_IR) fail(THM_EINVAL, "unknown precision");
    if (o->orth != THM_ORTH_CGS && o->orth != THM_ORTH_CGS2) fail(THM_EINVAL, "unknown orthogonalisation");
    if (o->krylov != THM_KRYLOV_COMPLEX && o->krylov != THM_KRYLOV_REAL) fail(THM_EINVAL, "unknown krylov kind");
    if (o->precond != THM_PREC_BLOCK && o->precond != THM_PREC_FULL) fail(THM_EINVAL, "unknown preconditioner");
    if (o->ir_mode != THM_IR_CLASSIC && o->ir_mode != THM_IR_GMRES) fail(THM_EINVAL, "unknown refinement mode");
}

thm_status thm_assemble(const thm_problem *p, void *stream, thm_system **out) {
    return guard([&] {
        if (!out) fail(THM_EINVAL, "out is NULL");
        *out = nullptr;
        validate(p);
        hipStream_t st = (hipStream_t)stream;
        auto S = std::make_unique<thm_system>();
        assemble_system(*S, *p, 0u, st);
        int nsub = 1;
        for (int a = 0; a < p->dim; ++a) nsub *= std::max(1, p->subdomains[a]);
        S->prob.subdomains[0] = std::max(1, p->subdomains[0]);
        S->prob.subdomains[1] = std::max(1, p->subdomains[1]);
        S->prob.subdomains[2] = p->dim == 3 ? std::max(1, p->subdomains[2]) : 1;
        (void)nsub;
        THM_HIP(hipStreamSynchronize(st));
        *out = S.release();
    });
}

thm_status thm_gmres_solve(int32_t nsys, thm_system *const *sys, const thm_solve_opts *opts, void *const *E_dev,
                           thm_stats *stats, void *stream) {
    int worst = THM_OK;
    thm_status rc = guard([&] {
        if (nsys < 1 || !sys || !E_dev || !stats) fail(THM_EINVAL, "bad arguments");
        check_opts(opts);
        for (int i = 0; i < nsys; ++i)
            if (!sys[i] || !E_dev[i]) fail(THM_EINVAL, "NULL system or vector");
        hipStream_t us = (hipStream_t)stream;
        std::vector<std::vector<thm_system *>> groups;
        if (opts->batched) groups.push_back(std::vector<thm_system *>(sys, sys + nsys));
        else
            for (int i = 0; i < nsys; ++i) groups.push_back({sys[i]});
        int base = 0;
        for (auto &grp : groups) {
            const double t0 = now_ms();
            Ctx &c = get_ctx(grp, opts->restart);
            const double t1 = now_ms();
            stream_join(us, c.st);
            const int ns = (int)grp.size();
            for (int s = 0; s < ns; ++s) {
                c.copy_in(s, grp[s]->rhs.p, c.b64.p);
                c.copy_in(s, (const double *)E_dev[base + s], c.x64.p);
            }
            launch_zero_flagged<double>(c.K.B, c.dirs.p, c.x64.p, c.st);
            std::vector<int> it, rf;
            std::vector<double> rs;
            c.solve(*opts, opts->transpose ? -1.f : 1.f, nullptr, it, rf, rs);
            for (int s = 0; s < ns; ++s) {
                launch_expand_dirichlet(grp[s]->n, grp[s]->dir_d.p, grp[s]->gD.p, c.x64.p + c.K.B.h_off[s], c.st);
                c.copy_out(s, c.x64.p, (double *)E_dev[base + s]);
            }
            stream_join(c.st, us);
            THM_HIP(hipStreamSynchronize(us));
            const double t2 = now_ms();
            for (int s = 0; s < ns; ++s) {
                thm_stats &o = stats[base + s];
                o.iters = it[s];
                o.outer_iters = 0;
                o.refinements = rf[s];
                o.fp64_fallback = c.last_fb[s];
                o.gmres_ir = c.last_ir[s];
                o.precond_extra_bytes = opts->precond == THM_PREC_FULL ? c.full.bytes : 0;
                o.rel_residual = rs[s];
                o.status = (rs[s] <= opts->rtol) ? THM_OK : THM_NOT_CONVERGED;
                o.setup_ms = (grp[s]->fac ? grp[s]->fac->setup_ms : 0.0) + (t1 - t0);
                o.solve_ms = t2 - t1;
                worst = std::max(worst, (int)o.status);
            }
            base += ns;
        }
    });
    if (rc != THM_OK) return rc;
    if (worst == THM_NOT_CONVERGED) g_last_error = "GMRES did not reach rtol for at least one system";
    return (thm_status)worst;
}

thm_status thm_ddm_solve(thm_system *sys, const thm_solve_opts *opts, void *E_dev, thm_stats *stats, void *stream) {
    thm_status rc = guard([&] {
        if (!sys || !E_dev || !stats) fail(THM_EINVAL, "bad arguments");
        check_opts(opts);
        if (opts->max_outer < 1) fail(THM_EINVAL, "max_outer must be >= 1");
        hipStream_t us = (hipStream_t)stream;
        THM_HIP(hipStreamSynchronize(us));
        if (!sys->ddm) build_ddm(*sys, us);
        ddm_solve_impl(*sys, *opts, (double *)E_dev, *stats, us);
        THM_HIP(hipStreamSynchronize(us));
    });
    if (rc != THM_OK) return rc;
    if (stats->status == THM_NOT_CONVERGED) g_last_error = "DDM did not reach rtol";
    return (thm_status)stats->status;
}

thm_status thm_adjoint_grad(thm_system *sys, const void *E_dev, const double tgt_lo[3], const double tgt_hi[3],
                            const thm_solve_opts *opts, double *dJdmu_dev, double *J_host, void *stream) {
    return guard([&] {
        if (!sys || !E_dev || !tgt_lo || !tgt_hi || !dJdmu_dev || !J_host) fail(THM_EINVAL, "bad arguments");
        check_opts(opts);
        thm_system &S = *sys;
        const Topo &t = S.topo;
        hipStream_t us = (hipStream_t)stream;
        Ctx &c = get_ctx({sys}, opts->restart);
        stream_join(us, c.st);
        DBuf<double> tl(3), th(3), rc((size_t)t.n_cells * t.n_loc * 2), Jc(t.n_cells), J(1);
        THM_HIP(hipMemcpyAsync(tl.p, tgt_lo, 3 * sizeof(double), hipMemcpyHostToDevice, c.st));
        THM_HIP(hipMemcpyAsync(th.p, tgt_hi, 3 * sizeof(double), hipMemcpyHostToDevice, c.st));
        launch_target_rhs(t.dim, t.p, t.n_cells, t.n_loc, S.fns.p, S.cell_dofs.p, S.h.p, S.lo.p, S.ncell.p, tl.p, th.p,
                          (const double *)E_dev, S.dir_d.p, rc.p, Jc.p, c.st);
        launch_sum(Jc.p, t.n_cells, J.p, c.st);
        launch_gather_vec(S.n, S.d2c_ptr.p, S.d2c_src.p, rc.p, c.b64.p, c.st);
        launch_zero_flagged<double>(c.K.B, c.dirs.p, c.b64.p, c.st);
        THM_HIP(hipMemsetAsync(c.x64.p, 0, sizeof(double) * c.x64.n, c.st));
        std::vector<int> it, rf;
        std::vector<double> rs;
        c.solve(*opts, -1.f, nullptr, it, rf, rs);
        launch_cell_gradient(t.dim, t.n_cells, t.n_loc, S.tcell, S.cell_dofs.p, S.h.p, S.mu_d.p,
                             (const double *)E_dev, c.x64.p, dJdmu_dev, c.st);
        THM_HIP(hipMemcpyAsync(J_host, J.p, sizeof(double), hipMemcpyDeviceToHost, c.st));
        THM_HIP(hipStreamSynchronize(c.st));
        stream_join(c.st, us);
        if (!(rs[0] <= opts->rtol)) fail(THM_NOT_CONVERGED, "adjoint solve did not reach rtol");
    });
}

thm_status thm_system_info(const thm_system *sys, thm_info *info) {
    return guard([&] {
        if (!sys || !info) fail(THM_EINVAL, "bad arguments");
        info->n_dofs = sys->n;
        info->n_free = sys->n_free;
        info->nnz = (int64_t)sys->K.col.size();
        info->nnz_c = (int64_t)sys->C.col.size();
        info->n_cells = sys->topo.n_cells;
        info->n_subdomains = sys->prob.subdomains[0] * sys->prob.subdomains[1] * sys->prob.subdomains[2];
        info->n_layers = sys->L.nlayers;
        info->factor_bytes = sys->fac ? sys->fac->bytes : -1;
        info->n_interface = sys->ddm ? sys->ddm->nent : -1;
        info->spmv_variant = -1;
        info->ddm_spmv_variant = -1;
        info->ddm_spmv_groups = -1;
        if (sys->ddm && sys->ddm->inner) {
            info->ddm_spmv_variant = sys->ddm->inner->lpr64;
            info->ddm_spmv_groups = sys->ddm->inner->ngroups;
        }
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            auto it = g_ctx_cache.find(std::vector<thm_system *>{const_cast<thm_system *>(sys)});
            if (it != g_ctx_cache.end() && it->second) info->spmv_variant = it->second->lpr64;
        }
    });
}

thm_status thm_system_release_workspaces(thm_system *sys) {
    return guard([&] {
        if (!sys) fail(THM_EINVAL, "bad arguments");
        drop_contexts(sys);
        for (auto &s : sys->subs) drop_contexts(s.get());
    });
}

thm_status thm_system_set_mu(thm_system *sys, const double *mu_dev, void *stream) {
    return guard([&] {
        if (!sys || !mu_dev) fail(THM_EINVAL, "bad arguments");
        if (sys->prob.subdomains[0] * sys->prob.subdomains[1] * sys->prob.subdomains[2] > 1)
            fail(THM_EUNSUPPORTED, "set_mu on a partitioned system");
        hipStream_t st = (hipStream_t)stream;
        std::vector<double> h(sys->topo.n_cells);
        THM_HIP(hipMemcpyAsync(h.data(), mu_dev, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
        THM_HIP(hipStreamSynchronize(st));
        for (double v : h)
            if (!(v > 0.0) || !std::isfinite(v)) fail(THM_EINVAL, "mu must be finite and > 0");
        drop_contexts(sys);
        sys->mu_host = h;
        THM_HIP(hipMemcpyAsync(sys->mu_d.p, mu_dev, sizeof(double) * h.size(), hipMemcpyDeviceToDevice, st));
        assemble_K(*sys, st);
        compute_lift(*sys, st);
        sys->fac.reset();
        for (auto &s : sys->subs) s->fac.reset();
        THM_HIP(hipStreamSynchronize(st));
    });
}

void thm_system_destroy(thm_system *sys) {
    if (!sys) return;
    try {
        drop_contexts(sys);
        for (auto &s : sys->subs) drop_contexts(s.get());
        if (sys->ddm) {
            sys->ddm->inner.reset();
            sys->ddm->singles.clear();
        }
        (void)hipDeviceSynchronize();
        delete sys;
    } catch (...) {
    }
}

thm_status thm_apply_operator(thm_system *sys, int32_t transpose, int32_t precision, const void *x_dev, void *y_dev,
                              void *stream) {
    return guard([&] {
        if (!sys || !x_dev || !y_dev) fail(THM_EINVAL, "bad arguments");
        hipStream_t us = (hipStream_t)stream;
        Ctx &c = get_ctx({sys}, 50);
        stream_join(us, c.st);
        c.copy_in(0, (const double *)x_dev, c.x64.p);
        const float sg = transpose ? -1.f : 1.f;
        if (precision == THM_FP32_IR) {
            KOps<float> o = c.ops32(sg, false);
            launch_scale<double, float>(c.K.B, nullptr, nullptr, 0, c.x64.p, c.x32.p, nullptr, 0, nullptr, c.st);
            o.apply(c.x32.p, c.b32.p, nullptr, nullptr);
            launch_scale<float, double>(c.K.B, nullptr, nullptr, 0, c.b32.p, c.r64.p, nullptr, 0, nullptr, c.st);
        } else {
            c.ops64(sg, false).apply(c.x64.p, c.r64.p, nullptr, nullptr);
        }
        c.copy_out(0, c.r64.p, (double *)y_dev);
        stream_join(c.st, us);
        THM_HIP(hipStreamSynchronize(us));
    });
}

thm_status thm_apply_precond(thm_system *sys, int32_t precision, const void *x_dev, void *y_dev, void *stream) {
    return guard([&] {
        if (!sys || !x_dev || !y_dev) fail(THM_EINVAL, "bad arguments");
        hipStream_t us = (hipStream_t)stream;
        Ctx &c = get_ctx({sys}, 50);
        stream_join(us, c.st);
        c.copy_in(0, (const double *)x_dev, c.x64.p);
        if (precision == THM_FP32_IR) {
            KOps<float> o = c.ops32(1.f);
            launch_scale<double, float>(c.K.B, nullptr, nullptr, 0, c.x64.p, c.x32.p, nullptr, 0, nullptr, c.st);
            o.prec(c.x32.p, c.b32.p, nullptr);
            launch_scale<float, double>(c.K.B, nullptr, nullptr, 0, c.b32.p, c.r64.p, nullptr, 0, nullptr, c.st);
        } else {
            c.ops64(1.f).prec(c.x64.p, c.r64.p, nullptr);
        }
        c.copy_out(0, c.r64.p, (double *)y_dev);
        stream_join(c.st, us);
        THM_HIP(hipStreamSynchronize(us));
    });
}

thm_status thm_apply_precond_noalloc(thm_system *sys, int32_t precision, const void *x_dev, void *y_dev,
                                     void *stream) {
    return guard([&] {
        if (!sys || !x_dev || !y_dev) fail(THM_EINVAL, "bad arguments");
        if (precision != THM_FP64 && precision != THM_FP32_IR) fail(THM_EINVAL, "unknown precision");
        // the system's own single-system context (looked up, never created: no allocation)
        Ctx *c = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            for (auto &kv : g_ctx_cache)
                if (kv.first.size() == 1 && kv.first[0] == sys && kv.second) c = kv.second.get();
        }
        if (!c || !c->prec_ready)
            fail(THM_EINVAL, "preconditioner of this system not built yet: call thm_apply_precond once first");
        noalloc_prec_apply(*c, precision, (const double *)x_dev, (double *)y_dev, (hipStream_t)stream);
    });
}

thm_status thm_apply_precond_full(thm_system *sys, int32_t transpose, int32_t precision, const void *x_dev,
                                  void *y_dev, void *stream) {
    return guard([&] {
        if (!sys || !x_dev || !y_dev) fail(THM_EINVAL, "bad arguments");
        hipStream_t us = (hipStream_t)stream;
        Ctx &c = get_ctx({sys}, 50);
        stream_join(us, c.st);
        c.copy_in(0, (const double *)x_dev, c.x64.p);
        const float cs = transpose ? -1.f : 1.f;
        if (precision == THM_FP32_IR) {
            KOps<float> o = c.ops32(cs, true, 1);
            launch_scale<double, float>(c.K.B, nullptr, nullptr, 0, c.x64.p, c.x32.p, nullptr, 0, nullptr, c.st);
            o.prec(c.x32.p, c.b32.p, nullptr);
            launch_scale<float, double>(c.K.B, nullptr, nullptr, 0, c.b32.p, c.r64.p, nullptr, 0, nullptr, c.st);
        } else {
            c.ops64(cs, true, 1).prec(c.x64.p, c.r64.p, nullptr);
        }
        c.copy_out(0, c.r64.p, (double *)y_dev);
        stream_join(c.st, us);
        THM_HIP(hipStreamSynchronize(us));
    });
}

thm_status thm_export_matrices(thm_system *sys, int32_t *k_rowptr, int32_t *k_col, double *k_val, int32_t *c_rowptr,
                               int32_t *c_col, double *c_val) {
    return guard([&] {
        if (!sys) fail(THM_EINVAL, "bad arguments");
        const thm_system &S = *sys;
        if (k_rowptr) std::copy(S.K.rowptr.begin(), S.K.rowptr.end(), k_rowptr);
        if (k_col) std::copy(S.K.col.begin(), S.K.col.end(), k_col);
        if (k_val) THM_HIP(hipMemcpy(k_val, S.kraw.p, sizeof(double) * S.K.col.size(), hipMemcpyDeviceToHost));
        if (c_rowptr) std::copy(S.C.rowptr.begin(), S.C.rowptr.end(), c_rowptr);
        if (c_col) std::copy(S.C.col.begin(), S.C.col.end(), c_col);
        if (c_val && !S.C.col.empty())
            THM_HIP(hipMemcpy(c_val, S.craw.p, sizeof(double) * S.C.col.size(), hipMemcpyDeviceToHost));
    });
}

thm_status thm_export_rhs(thm_system *sys, uint8_t *dir_flags, double *gD, double *rhs) {
    return guard([&] {
        if (!sys) fail(THM_EINVAL, "bad arguments");
        const thm_system &S = *sys;
        if (dir_flags) std::copy(S.dir.begin(), S.dir.end(), dir_flags);
        if (gD) THM_HIP(hipMemcpy(gD, S.gD.p, sizeof(double) * 2 * S.n, hipMemcpyDeviceToHost));
        if (rhs) THM_HIP(hipMemcpy(rhs, S.rhs.p, sizeof(double) * 2 * S.n, hipMemcpyDeviceToHost));
    });
}

thm_status thm_export_elements(thm_system *sys, int64_t c0, int64_t count, double *out) {
    return guard([&] {
        if (!sys || !out || c0 < 0 || count < 0 || c0 + count > sys->topo.n_cells) fail(THM_EINVAL, "bad arguments");
        const int64_t nl2 = (int64_t)sys->topo.n_loc * sys->topo.n_loc;
        THM_HIP(hipMemcpy(out, sys->kel.p + c0 * nl2, sizeof(double) * count * nl2, hipMemcpyDeviceToHost));
    });
}

thm_status thm_time_spmv(thm_system *sys, int32_t precision, int32_t reps, double *ms_out, double *bytes_out,
                         void *stream) {
    return guard([&] {
        if (!sys || !ms_out || reps < 1) fail(THM_EINVAL, "bad arguments");
        hipStream_t us = (hipStream_t)stream;
        Ctx &c = get_ctx({sys}, 50);
        stream_join(us, c.st);
        hipEvent_t e0, e1;
        THM_HIP(hipEventCreate(&e0));
        THM_HIP(hipEventCreate(&e1));
        const bool f32 = precision == THM_FP32_IR;
        KOps<double> o64 = c.ops64(1.f, false);
        KOps<float> o32 = c.ops32(1.f, false);
        auto once = [&] {
            if (f32) o32.apply(c.x32.p, c.b32.p, nullptr, nullptr);
            else o64.apply(c.x64.p, c.r64.p, nullptr, nullptr);
        };
        once();
        THM_HIP(hipEventRecord(e0, c.st));
        for (int r = 0; r < reps; ++r) once();
        THM_HIP(hipEventRecord(e1, c.st));
        THM_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        THM_HIP(hipEventElapsedTime(&ms, e0, e1));
        THM_HIP(hipEventDestroy(e0));
        THM_HIP(hipEventDestroy(e1));
        *ms_out = ms / reps;
        const double v = f32 ? 4.0 : 8.0;
        const double nnz = (double)sys->K.col.size() + (double)sys->C.col.size();
        if (bytes_out) *bytes_out = (v + 4.0) * nnz + 2.0 * 4.0 * (sys->n + 1) + 2.0 * 2.0 * sys->n * v;
        stream_join(c.st, us);
    });
}

thm_status thm_time_spmv_batch(thm_system *sys, int32_t precision, int32_t variant, int32_t reps, double *ms_out,
                               double *bytes_out, void *stream) {
    return guard([&] {
        if (!sys || !ms_out || reps < 1) fail(THM_EINVAL, "bad arguments");
        if (precision != THM_FP64 && precision != THM_FP32_IR) fail(THM_EINVAL, "unknown precision");
        if (!sys->ddm || !sys->ddm->inner) fail(THM_EINVAL, "no subdomain batch yet: run thm_ddm_solve first");
        static const int known[] = {21, 41, 81, 161, 321, 641, 24, 44, 84, 164, 324, THM_SPMV_SELL,
                                    THM_SPMV_SELL_GROUP, THM_SPMV_SELL_GROUP_IL};
        bool ok = variant == -1;
        for (int k : known) ok = ok || k == variant;
        if (!ok) fail(THM_EINVAL, "unknown SpMV variant");
        Ctx &c = *sys->ddm->inner;
        const bool f32 = precision == THM_FP32_IR;
        const int v = variant >= 0 ? variant : (f32 ? c.lpr32 : c.lpr64);
        hipStream_t us = (hipStream_t)stream;
        stream_join(us, c.st);
        c.ops32(1.f, false);  // allocates the FP32 slots on first use
        hipEvent_t e0, e1;
        THM_HIP(hipEventCreate(&e0));
        THM_HIP(hipEventCreate(&e1));
        if (v == THM_SPMV_SELL_GROUP_IL) c.ensure_xi(f32);
        auto once = [&] {
            if (v == THM_SPMV_SELL_GROUP_IL) {
                if (f32)
                    launch_spmv_group_i<float>(c.mat32.p, c.K.B.off.p, c.sgroups.p, c.gsched, c.ngroups, nullptr,
                                               c.xi32.p, c.b32.p, 1.f, c.st);
                else
                    launch_spmv_group_i<double>(c.mat64.p, c.K.B.off.p, c.sgroups.p, c.gsched, c.ngroups, nullptr,
                                                c.xi64.p, c.r64.p, 1.f, c.st);
                return;
            }
            if (f32) c.spmv<float>(v, nullptr, c.x32.p, c.b32.p, nullptr, 1.f);
            else c.spmv<double>(v, nullptr, c.x64.p, c.r64.p, nullptr, 1.f);
        };
        once();
        THM_HIP(hipEventRecord(e0, c.st));
        for (int r = 0; r < reps; ++r) once();
        THM_HIP(hipEventRecord(e1, c.st));
        THM_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        THM_HIP(hipEventElapsedTime(&ms, e0, e1));
        THM_HIP(hipEventDestroy(e0));
        THM_HIP(hipEventDestroy(e1));
        *ms_out = ms / reps;
        if (bytes_out) {
            const double w = f32 ? 4.0 : 8.0;
            double by = 0.0;
            for (const SpmvGroup &g : c.hgroups) {  // each distinct K once, with its row pointers
                const thm_system &R = *c.sys[g.rep];
                by += (w + 4.0) * (double)R.K.col.size() + 4.0 * (double)(R.n + 1);
            }
            for (const thm_system *m : c.sys)  // per system: C, its row pointers, x read and y written
                by += (w + 4.0) * (double)m->C.col.size() + 4.0 * (double)(m->n + 1) + 2.0 * 2.0 * m->n * w;
            *bytes_out = by;
        }
        stream_join(c.st, us);
    });
}

thm_status thm_time_spmv_systems(int32_t nsys, thm_system *const *sys, int32_t precision, int32_t reps,
                                 double *ms_out, double *bytes_out, void *stream) {
    return guard([&] {
        if (nsys < 1 || !sys || !ms_out || reps < 1) fail(THM_EINVAL, "bad arguments");
        if (precision != THM_FP64 && precision != THM_FP32_IR) fail(THM_EINVAL, "unknown precision");
        std::vector<thm_system *> grp(sys, sys + nsys);
        for (thm_system *s : grp)
            if (!s) fail(THM_EINVAL, "NULL system");
        Ctx *c = nullptr;
        {
            // the batch context of an earlier thm_gmres_solve on the same systems, whatever its restart
            std::lock_guard<std::mutex> lk(g_cache_mu);
            auto it = g_ctx_cache.find(grp);
            if (it != g_ctx_cache.end() && it->second) c = it->second.get();
        }
        if (!c) c = &get_ctx(grp, 50);
        const bool f32 = precision == THM_FP32_IR;
        hipStream_t us = (hipStream_t)stream;
        stream_join(us, c->st);
        c->ops32(1.f, false);  // allocates the FP32 slots on first use
        const int v = f32 ? c->lpr32 : c->lpr64;
        hipEvent_t e0, e1;
        THM_HIP(hipEventCreate(&e0));
        THM_HIP(hipEventCreate(&e1));
        auto once = [&] {
            if (f32) c->spmv<float>(v, nullptr, c->x32.p, c->b32.p, nullptr, 1.f);
            else c->spmv<double>(v, nullptr, c->x64.p, c->r64.p, nullptr, 1.f);
        };
        once();
        THM_HIP(hipEventRecord(e0, c->st));
        for (int r = 0; r < reps; ++r) once();
        THM_HIP(hipEventRecord(e1, c->st));
        THM_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        THM_HIP(hipEventElapsedTime(&ms, e0, e1));
        THM_HIP(hipEventDestroy(e0));
        THM_HIP(hipEventDestroy(e1));
        *ms_out = ms / reps;
        if (bytes_out) {
            const double w = f32 ? 4.0 : 8.0;
            double by = 0.0;
            if (v == THM_SPMV_SELL_GROUP)
                for (const SpmvGroup &g : c->hgroups) {  // each distinct K once, with its row pointers
                    const thm_system &R = *c->sys[g.rep];
                    by += (w + 4.0) * (double)R.K.col.size() + 4.0 * (double)(R.n + 1);
                }
            for (const thm_system *m : c->sys) {
                if (v != THM_SPMV_SELL_GROUP) by += (w + 4.0) * (double)m->K.col.size() + 4.0 * (double)(m->n + 1);
                by += (w + 4.0) * (double)m->C.col.size() + 4.0 * (double)(m->n + 1) + 2.0 * 2.0 * m->n * w;
            }
            *bytes_out = by;
        }
        stream_join(c->st, us);
    });
}

static_assert(THM_NOALLOC_SCRATCH_BYTES == thm::NOALLOC_SCRATCH_BYTES, "scratch size of the header and the library");
static_assert(THM_SPMV_SELL_GROUP_IL == thm::SPMV_SELL_GROUP_IL, "interleaved grouped SpMV code");
static_assert(THM_SPMV_SELL == thm::SPMV_SELL && THM_SPMV_SELL_GROUP == thm::SPMV_SELL_GROUP,
              "SpMV variant codes of the header and the kernels differ");

thm_status thm_set_spmv_variant(thm_system *sys, int32_t precision, int32_t variant) {
    return guard([&] {
        if (!sys) fail(THM_EINVAL, "bad arguments");
        if (precision != THM_FP64 && precision != THM_FP32_IR) fail(THM_EINVAL, "unknown precision");
        static const int known[] = {21, 41, 81, 161, 321, 641, 24, 44, 84, 164, 324, THM_SPMV_SELL,
                                    THM_SPMV_SELL_GROUP, THM_SPMV_SELL_GROUP_IL};
        bool ok = variant == -1;
        for (int k : known) ok = ok || k == variant;
        if (!ok) fail(THM_EINVAL, "unknown SpMV variant");
        auto pin = [&](Ctx &c) {
            c.K.drop_graphs();  // captured steps hold the previous variant's kernel
            if (variant == -1) {
                c.autotune();
                return;
            }
            if (variant != THM_SPMV_SELL_GROUP && variant != THM_SPMV_SELL_GROUP_IL) c.K.B.spmv_sched(variant, c.st);
            if (precision == THM_FP64) c.lpr64 = variant;
            else c.lpr32 = variant;
        };
        pin(get_ctx({sys}, 50));
        if (sys->ddm && sys->ddm->inner) pin(*sys->ddm->inner);
    });
}

thm_status thm_time_precond(thm_system *sys, int32_t precision, int32_t reps, double *ms_out, double *bytes_out,
                            int32_t *launches_out, void *stream) {
    return guard([&] {
        if (!sys || !ms_out || reps < 1) fail(THM_EINVAL, "bad arguments");
        hipStream_t us = (hipStream_t)stream;
        Ctx *c = nullptr;
        if (sys->ddm && sys->ddm->inner) c = sys->ddm->inner.get();
        else c = &get_ctx({sys}, 50);
        stream_join(us, c->st);
        double by = 0.0;
        int nl = 0;
        *ms_out = c->time_bcr(precision == THM_FP32_IR ? 1 : 0, reps, &by, &nl);
        if (bytes_out) *bytes_out = by;
        if (launches_out) *launches_out = nl;
        stream_join(c->st, us);
    });
}

}  // extern "C"
