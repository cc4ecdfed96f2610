// Setup of the block preconditioner diag(K, K)^{-1} (eq. (11)) as an exact
// factorised K^{-1}: static condensation of cell interiors, then block cyclic
// reduction over the layers of skeleton DoFs (thin layers), or block LU (thick layers,
// see plan_lu).  The paper approximates K^{-1} by an AMG with direct level transitions;
// here the inverse is exact, so GMRES sees the preconditioned operator
// I + [[0, -K^{-1}C], [K^{-1}C, 0]].
//
// Cyclic reduction on the block-tridiagonal skeleton matrix (diagonal blocks D_i,
// couplings Lo_i between position i and i-1): at every level the odd positions p
// are eliminated with explicit inverses Dinv_p; each even position q keeps
//   Gm_q = Lo_q Dinv_{q-1},  Gp_q = Lo_{q+1}^T Dinv_{q+1},
//   D_q <- D_q - Gm_q Lo_q^T - Gp_q Lo_{q+1},  Lo_q <- -Gm_q Lo_{q-1}.
// Application: reduce the right-hand side upwards (r_q -= Gm_q r_{q-1} + Gp_q r_{q+1}),
// solve the last block, then substitute downwards
// (x_p = Dinv_p r_p - Gp_{p-1}^T x_{p-1} - Gm_{p+1}^T x_{p+1}).
// Systems whose Dirichlet-modified K and element matrices are bitwise identical
// share one factor.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>

#include "solver.h"

namespace thm {

static bool same_topology(const thm_system &a, const thm_system &b) {
    const Topo &x = a.topo, &y = b.topo;
    if (x.dim != y.dim || x.p != y.p) return false;
    for (int i = 0; i < 3; ++i)
        if (x.n[i] != y.n[i] || x.h[i] != y.h[i]) return false;
    return a.K.col.size() == b.K.col.size() && a.dir == b.dir;
}

static bool same_values(thm_system &a, thm_system &b, hipStream_t st) {
    DBuf<int32_t> flag(1);
    THM_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), st));
    launch_compare(a.kval.p, b.kval.p, (int64_t)a.K.col.size(), flag.p, st);
    launch_compare(a.kel.p, b.kel.p, (int64_t)a.kel.n, flag.p, st);
    int32_t h = 1;
    THM_HIP(hipMemcpyAsync(&h, flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    THM_HIP(hipStreamSynchronize(st));
    return h == 0;
}

bool same_matrices(thm_system &a, thm_system &b, hipStream_t st) {
    return same_topology(a, b) && a.K.rowptr == b.K.rowptr && a.K.col == b.K.col && same_values(a, b, st);
}

namespace {
// Work of one factor during setup.
struct Work {
    thm_system *rep;
    Factor *f;
    DBuf<double> D, Lo0;                  // initial diagonal / coupling blocks (layering offsets)
    std::map<int, DBuf<double>> lo;       // per layer: current coupling to the previous position (level > 0)
    std::vector<int> pos;
    const double *lo_ptr(int layer) const {
        auto it = lo.find(layer);
        if (it != lo.end()) return it->second.p;
        return Lo0.p + rep->L.lf_off[layer];
    }
    double *d_ptr(int layer) { return D.p + rep->L.sinv_off[layer]; }
};
}  // namespace

// Padded copies for the apply: each input segment starts at its layer's aligned width,
// the row length is padded to a multiple of the MFMA column step and the row count to a
// multiple of the row tile; stored tile by tile (see k_repack).
static void pad_blocks(Factor &f) {
    int64_t poff = 0;
    auto pad = [&](Factor::Blk &b) {
        int c = 0;
        for (int q = 0; q < b.nseg; ++q) {
            b.seg_pstart[q] = c;
            const int k = b.seg_layer[q];
            c += (int)(f.pboff[k + 1] - f.pboff[k]);
        }
        b.seg_pstart[b.nseg] = c;
        b.ld = (c + BCR_KS - 1) / BCR_KS * BCR_KS;
        if (b.ld > 8 * BCR_TAB)
            fail(THM_EUNSUPPORTED, "a factor block has more columns than the apply kernel supports");
        b.poff = poff;
        poff += (int64_t)(b.rows + BCR_RT - 1) / BCR_RT * BCR_RT * b.ld;
    };
    for (auto &lev : f.fwd)
        for (auto &b : lev) pad(b);
    for (auto &lev : f.bwd)
        for (auto &b : lev) pad(b);
    for (auto &b : f.tops) pad(b);
    f.matp_elems = poff;
}

// Plan the level structure of one factor and the offsets of its apply matrices.
static void plan(Factor &f) {
    const int nL = f.nlayers;
    std::vector<int> pos(nL);
    for (int k = 0; k < nL; ++k) pos[k] = k;
    int64_t off = 0;
    auto blk = [&](int layer, int cols) {
        Factor::Blk b{};
        b.layer = layer;
        b.rows = f.bsize[layer];
        b.cols = cols;
        b.off = off;
        off += (int64_t)b.rows * cols;
        return b;
    };
    f.fwd.clear();
    f.bwd.clear();
    f.fw_at.clear();
    f.bk_at.clear();
    f.level_pos.clear();
    auto total = [&](const std::vector<int> &v) {
        int64_t t = 0;
        for (int k : v) t += f.bsize[k];
        return t;
    };
    constexpr int TOP_BLOCKS = 9;
    constexpr int64_t TOP_ROWS = 6144;
    while (pos.size() > 1 && !((int)pos.size() <= TOP_BLOCKS && total(pos) <= TOP_ROWS)) {
        const int m = (int)pos.size();
        std::vector<Factor::Blk> fw, bk;
        std::map<int, int> fwi, bki;
        for (int i = 1; i < m; i += 2) {
            const int b = f.bsize[pos[i]];
            const int bl = f.bsize[pos[i - 1]];
            const int br = i + 1 < m ? f.bsize[pos[i + 1]] : 0;
            Factor::Blk x = blk(pos[i], b + bl + br);
            x.nseg = 0;
            x.seg_layer[x.nseg] = pos[i]; x.seg_src[x.nseg++] = 0;
            x.seg_layer[x.nseg] = pos[i - 1]; x.seg_src[x.nseg++] = 1;
            if (i + 1 < m) { x.seg_layer[x.nseg] = pos[i + 1]; x.seg_src[x.nseg++] = 1; }
            x.out_dst = 1;
            x.subtract = 0;
            bki[i] = (int)bk.size();
            bk.push_back(x);
        }
        for (int i = 0; i < m; i += 2) {
            const int bl = i > 0 ? f.bsize[pos[i - 1]] : 0;
            const int br = i + 1 < m ? f.bsize[pos[i + 1]] : 0;
            Factor::Blk x = blk(pos[i], bl + br);
            x.nseg = 0;
            if (i > 0) { x.seg_layer[x.nseg] = pos[i - 1]; x.seg_src[x.nseg++] = 0; }
            if (i + 1 < m) { x.seg_layer[x.nseg] = pos[i + 1]; x.seg_src[x.nseg++] = 0; }
            x.out_dst = 0;
            x.subtract = 1;
            fwi[i] = (int)fw.size();
            fw.push_back(x);
        }
        f.fwd.push_back(fw);
        f.bwd.push_back(bk);
        f.fw_at.push_back(fwi);
        f.bk_at.push_back(bki);
        f.level_pos.push_back(pos);
        std::vector<int> even;
        for (int i = 0; i < m; i += 2) even.push_back(pos[i]);
        pos = even;
    }
    // dense inverse of the remaining block-tridiagonal system, one task per block row
    f.top_pos = pos;
    f.top_n = (int)total(pos);
    f.top_off = off;
    f.tops.clear();
    int64_t roff = 0;
    for (int k : pos) {
        Factor::Blk b{};
        b.layer = k;
        b.rows = f.bsize[k];
        b.cols = f.top_n;
        b.off = f.top_off + roff * f.top_n;
        b.nseg = (int)pos.size();
        for (size_t q = 0; q < pos.size(); ++q) {
            b.seg_layer[q] = pos[q];
            b.seg_src[q] = 0;
        }
        b.out_dst = 1;
        b.subtract = 0;
        f.tops.push_back(b);
        roff += f.bsize[k];
    }
    off += (int64_t)f.top_n * f.top_n;
    f.mat_elems = off;
    pad_blocks(f);
}

// Plan of the block-LU form (thick layers): forward task i computes
//   y_i = S_i^{-1} r_i - (S_i^{-1} Lo_i) y_{i-1}        (matrix [S_i^{-1} | -S_i^{-1} Lo_i]),
// backward task i (from the last but one layer down) computes
//   x_i = y_i - (S_i^{-1} Lo_{i+1}^T) x_{i+1}          (subtracting task),
// with the block pivots S_0 = D_0, S_i = D_i - Lo_i S_{i-1}^{-1} Lo_i^T.  One forward and one
// backward level per layer, one task each; no dense last system.
static void plan_lu(Factor &f) {
    const int nL = f.nlayers;
    int64_t off = 0;
    f.fwd.clear();
    f.bwd.clear();
    f.fw_at.clear();
    f.bk_at.clear();
    f.level_pos.clear();
    f.tops.clear();
    f.top_pos.clear();
    f.top_n = 0;
    for (int i = 0; i < nL; ++i) {
        Factor::Blk b{};
        b.layer = i;
        b.rows = f.bsize[i];
        b.cols = f.bsize[i] + (i > 0 ? f.bsize[i - 1] : 0);
        b.off = off;
        off += (int64_t)b.rows * b.cols;
        b.nseg = 0;
        b.seg_layer[b.nseg] = i; b.seg_src[b.nseg++] = 0;
        if (i > 0) { b.seg_layer[b.nseg] = i - 1; b.seg_src[b.nseg++] = 1; }
        b.out_dst = 1;
        b.subtract = 0;
        f.fwd.push_back({b});
    }
    for (int i = 0; i + 1 < nL; ++i) {
        Factor::Blk b{};
        b.layer = i;
        b.rows = f.bsize[i];
        b.cols = f.bsize[i + 1];
        b.off = off;
        off += (int64_t)b.rows * b.cols;
        b.nseg = 0;
        b.seg_layer[b.nseg] = i + 1; b.seg_src[b.nseg++] = 1;
        b.out_dst = 1;
        b.subtract = 1;
        f.bwd.push_back({b});
    }
    f.top_off = off;
    f.mat_elems = off;
    pad_blocks(f);
}

// Cyclic reduction keeps about 5 b^2 words per layer of width b and applies them in
// 2 log2(layers) + 1 launches; block LU keeps 3 b^2 and needs 2 layers - 1 launches.  With
// few thick layers (3D subdomains: 9 layers of 1,282 at 8^3, 17 of 4,866 at 16^3) each
// block-LU launch is large enough to stream at full rate and block LU reads fewer bytes for
// the same K^{-1}; with many thin layers (2D meshes) the launches are latency-bound and the
// long chain of pivots is the less accurate one in FP32, so cyclic reduction stays.
// THM_FACTOR_FORM=bcr|lu overrides the choice (tests of both forms on small problems).
constexpr int LU_MIN_LAYER = 1024;
constexpr int LU_MAX_LAYERS = 64;
static bool use_block_lu(const Layering &L) {
    if (const char *e = std::getenv("THM_FACTOR_FORM")) {
        const std::string v(e);
        if (v == "lu") return true;
        if (v == "bcr") return false;
        fail(THM_EINVAL, "THM_FACTOR_FORM must be bcr or lu");
    }
    int64_t wide = 0;
    for (int32_t b : L.bsize) wide = std::max<int64_t>(wide, b);
    return wide >= LU_MIN_LAYER && L.nlayers <= LU_MAX_LAYERS;
}

void setup_precond(const std::vector<thm_system *> &all, hipStream_t st, bool share) {
    std::vector<thm_system *> need;
    for (thm_system *s : all)
        if (!s->fac) need.push_back(s);
    if (need.empty()) return;
    const double t0 = now_ms();
    // group identical systems
    std::vector<std::shared_ptr<Factor>> facs;
    std::vector<thm_system *> reps;
    for (thm_system *s : need) {
        bool found = false;
        if (share)
            for (size_t g = 0; g < reps.size() && !found; ++g)
                if (same_topology(*reps[g], *s) && same_values(*reps[g], *s, st)) {
                    s->fac = facs[g];
                    found = true;
                }
        if (found) continue;
        auto f = std::make_shared<Factor>();
        s->fac = f;
        facs.push_back(f);
        reps.push_back(s);
    }
    DBuf<int32_t> status(1);
    THM_HIP(hipMemsetAsync(status.p, 0, sizeof(int32_t), st));
    std::vector<Work> W(facs.size());
    int maxlev = 0, maxn_lu = 0;
    for (size_t g = 0; g < facs.size(); ++g) {
        thm_system &R = *reps[g];
        Factor &f = *facs[g];
        const Layering &L = R.L;
        const Topo &t = R.topo;
        f.nlayers = L.nlayers;
        f.bsize = L.bsize;
        f.boff = L.boff;
        f.pboff = L.pboff;
        f.sp = L.n_skel_pad;
        f.n_int = t.n_int;
        f.ne = t.n_loc - t.n_int;
        f.n_cells = t.n_cells;
        f.lu = use_block_lu(L);
        if (f.lu) {
            plan_lu(f);
            maxn_lu = std::max(maxn_lu, f.nlayers);
        } else {
            plan(f);
            maxlev = std::max(maxlev, (int)f.fwd.size());
        }
        W[g].rep = &R;
        W[g].f = &f;
        // condensation of cell interiors
        f.kiinv.alloc(std::max<int64_t>((int64_t)t.n_cells * t.n_int * t.n_int, 1));
        f.F.alloc(std::max<int64_t>((int64_t)t.n_cells * f.ne * t.n_int, 1));
        DBuf<double> kcond((size_t)t.n_cells * f.ne * f.ne);
        launch_condense((int)t.n_cells, t.n_loc, t.n_int, R.kel.p, R.cell_dofs.p, R.dir_d.p, f.kiinv.p, f.F.p,
                        kcond.p, status.p, st);
        // initial blocks D_k, Lo_k from the condensed element matrices
        W[g].D.alloc(L.sinv_total);
        W[g].Lo0.alloc(std::max<int64_t>(L.lf_total, 1));
        launch_fill(W[g].D.p, L.sinv_total, 0.0, st);
        launch_fill(W[g].Lo0.p, L.lf_total, 0.0, st);
        {
            DBuf<int64_t> ti;
            DBuf<int32_t> tk, tp, ts;
            ti.upload(L.tgt_index, st);
            tk.upload(L.tgt_kind, st);
            tp.upload(L.tgt_ptr, st);
            ts.upload(L.tgt_src, st);
            launch_tgt_gather((int64_t)L.tgt_index.size(), ti.p, tk.p, tp.p, ts.p, kcond.p, W[g].D.p, W[g].Lo0.p, st);
            DBuf<int32_t> skel, bs;
            DBuf<int64_t> bo, so;
            skel.upload(L.skel_dof, st);
            bs.upload(L.bsize, st);
            bo.upload(L.boff, st);
            so.upload(L.sinv_off, st);
            launch_dir_identity(L.n_skel, skel.p, R.dir_d.p, bo.p, so.p, bs.p, L.nlayers, W[g].D.p, st);
            THM_HIP(hipStreamSynchronize(st));
        }
        f.mat.alloc(std::max<int64_t>(f.mat_elems, 1));
        for (int k = 0; k < L.nlayers; ++k) W[g].pos.push_back(k);
    }
    DBuf<GemmDesc> gscr;
    Sched gsched;
    auto run_gemms = [&](const std::vector<GemmDesc> &g) {
        if (g.empty()) return;
        launch_gemm_batched(g, st, gscr, gsched);
        THM_HIP(hipStreamSynchronize(st));
    };
    // inversion scratch
    auto invert = [&](std::vector<std::pair<const double *, std::pair<double *, int>>> jobs, const std::vector<int> &ns) {
        if (jobs.empty()) return;
        int64_t tot = 0, totp = 0;
        for (int n : ns) { tot += 2 * (int64_t)n * n; totp += 2 * n; }
        DBuf<double> work(std::max<int64_t>(tot, 1));
        DBuf<int32_t> piv(std::max<int64_t>(totp, 1));
        std::vector<InvDesc> d;
        int64_t o = 0, op = 0;
        for (size_t j = 0; j < jobs.size(); ++j) {
            const int n = ns[j];
            double *A = work.p + o, *Wb = work.p + o + (int64_t)n * n;
            THM_HIP(hipMemcpyAsync(A, jobs[j].first, sizeof(double) * n * n, hipMemcpyDeviceToDevice, st));
            d.push_back({n, A, Wb, jobs[j].second.first, piv.p + op, jobs[j].second.second});
            o += 2 * (int64_t)n * n;
            op += 2 * n;
        }
        launch_invert_blocked(d, status.p, st);
    };
    const bool progress = std::getenv("THM_PROGRESS") != nullptr;
    if (progress)
        std::fprintf(stderr, "[thm] preconditioner setup: %zu systems, %zu factors, %d levels, %.1f ms\n", need.size(),
                     facs.size(), maxlev, now_ms() - t0);
    for (int lev = 0; lev < maxlev; ++lev) {
        if (progress) std::fprintf(stderr, "[thm]   level %d at %.1f ms\n", lev, now_ms() - t0);
        std::vector<std::pair<const double *, std::pair<double *, int>>> jobs;
        std::vector<int> jn;
        std::vector<GemmDesc> gA, gB1, gB2;
        struct LoNew { Work *w; int layer; DBuf<double> buf; };
        std::vector<LoNew> lonew;
        // 1. inverses of the odd positions (into the first columns of their back-substitution blocks)
        for (Work &w : W) {
            Factor &f = *w.f;
            if (f.lu || lev >= (int)f.fwd.size()) continue;
            const auto &pos = f.level_pos[lev];
            for (int i = 1; i < (int)pos.size(); i += 2) {
                const Factor::Blk &b = f.bwd[lev][f.bk_at[lev].at(i)];
                jobs.push_back({w.d_ptr(pos[i]), {f.mat.p + b.off, b.cols}});
                jn.push_back(b.rows);
            }
        }
        invert(jobs, jn);
        // 2. Gm, Gp; 3. D updates and new couplings
        for (Work &w : W) {
            Factor &f = *w.f;
            if (f.lu || lev >= (int)f.fwd.size()) continue;
            const auto &pos = f.level_pos[lev];
            const int m = (int)pos.size();
            for (int i = 0; i < m; i += 2) {
                const Factor::Blk &fb = f.fwd[lev][f.fw_at[lev].at(i)];
                const int bq = f.bsize[pos[i]];
                double *Fw = f.mat.p + fb.off;
                int cofs = 0;
                if (i > 0) {
                    const int bl = f.bsize[pos[i - 1]];
                    const Factor::Blk &bkl = f.bwd[lev][f.bk_at[lev].at(i - 1)];
                    gA.push_back({bq, bl, bl, 0, 0, w.lo_ptr(pos[i]), f.mat.p + bkl.off, Fw, bl, bkl.cols, fb.cols,
                                  1.0, 0.0});
                    gB1.push_back({bq, bq, bl, 0, 1, Fw, w.lo_ptr(pos[i]), w.d_ptr(pos[i]), fb.cols, bl, bq, -1.0, 1.0});
                    if (i >= 2) {
                        const int bll = f.bsize[pos[i - 2]];
                        lonew.push_back({&w, pos[i], DBuf<double>((size_t)bq * bll)});
                        gB1.push_back({bq, bll, bl, 0, 0, Fw, w.lo_ptr(pos[i - 1]), lonew.back().buf.p, fb.cols, bll,
                                       bll, -1.0, 0.0});
                    }
                    cofs = bl;
                }
                if (i + 1 < m) {
                    const int br = f.bsize[pos[i + 1]];
                    const Factor::Blk &bkr = f.bwd[lev][f.bk_at[lev].at(i + 1)];
                    // Gp = Lo_{i+1}^T Dinv_{i+1}; Lo_{i+1} is br x bq
                    gA.push_back({bq, br, br, 1, 0, w.lo_ptr(pos[i + 1]), f.mat.p + bkr.off, Fw + cofs, bq, bkr.cols,
                                  fb.cols, 1.0, 0.0});
                    gB2.push_back({bq, bq, br, 0, 0, Fw + cofs, w.lo_ptr(pos[i + 1]), w.d_ptr(pos[i]), fb.cols, bq, bq,
                                   -1.0, 1.0});
                }
            }
        }
        run_gemms(gA);
        run_gemms(gB1);
        run_gemms(gB2);
        // 4. back-substitution couplings: -Gp_{p-1}^T and -Gm_{p+1}^T next to Dinv_p
        for (Work &w : W) {
            Factor &f = *w.f;
            if (f.lu || lev >= (int)f.fwd.size()) continue;
            const auto &pos = f.level_pos[lev];
            const int m = (int)pos.size();
            for (int i = 1; i < m; i += 2) {
                const Factor::Blk &b = f.bwd[lev][f.bk_at[lev].at(i)];
                const int bp = f.bsize[pos[i]], bl = f.bsize[pos[i - 1]];
                const Factor::Blk &fl = f.fwd[lev][f.fw_at[lev].at(i - 1)];
                const int lcofs = (i - 1 > 0) ? f.bsize[pos[i - 2]] : 0;  // Gp part of Fw_{i-1}
                launch_transpose(f.mat.p + fl.off + lcofs, bl, bp, fl.cols, f.mat.p + b.off + bp, b.cols, -1.0, st);
                if (i + 1 < m) {
                    const Factor::Blk &fr = f.fwd[lev][f.fw_at[lev].at(i + 1)];
                    const int br = f.bsize[pos[i + 1]];
                    launch_transpose(f.mat.p + fr.off, br, bp, fr.cols, f.mat.p + b.off + bp + bl, b.cols, -1.0, st);
                }
            }
        }
        THM_HIP(hipStreamSynchronize(st));
        for (LoNew &ln : lonew) ln.w->lo[ln.layer] = std::move(ln.buf);
    }
    // block LU, one layer at a time over every block-LU factor
    for (int i = 0; i < maxn_lu; ++i) {
        if (progress) std::fprintf(stderr, "[thm]   block-LU layer %d at %.1f ms\n", i, now_ms() - t0);
        std::vector<GemmDesc> ga, gb, gd;
        std::vector<std::pair<const double *, std::pair<double *, int>>> jobs;
        std::vector<int> jn;
        for (Work &w : W) {
            Factor &f = *w.f;
            if (!f.lu || i >= f.nlayers || i == 0) continue;
            const int b = f.bsize[i], bl = f.bsize[i - 1];
            const Factor::Blk &fl = f.fwd[i - 1][0], &bk = f.bwd[i - 1][0];
            // backward matrix of layer i-1: S_{i-1}^{-1} Lo_i^T (Lo_i is b x bl)
            ga.push_back({bl, b, bl, 0, 1, f.mat.p + fl.off, w.lo_ptr(i), f.mat.p + bk.off, fl.cols, bl, b, 1.0, 0.0});
            // pivot S_i = D_i - Lo_i (S_{i-1}^{-1} Lo_i^T)
            gb.push_back({b, b, bl, 0, 0, w.lo_ptr(i), f.mat.p + bk.off, w.d_ptr(i), bl, b, b, -1.0, 1.0});
        }
        run_gemms(ga);
        run_gemms(gb);
        for (Work &w : W) {
            Factor &f = *w.f;
            if (!f.lu || i >= f.nlayers) continue;
            const Factor::Blk &fb = f.fwd[i][0];
            jobs.push_back({w.d_ptr(i), {f.mat.p + fb.off, fb.cols}});
            jn.push_back(fb.rows);
        }
        invert(jobs, jn);
        THM_HIP(hipStreamSynchronize(st));
        for (Work &w : W) {
            Factor &f = *w.f;
            if (!f.lu || i >= f.nlayers || i == 0) continue;
            const int b = f.bsize[i], bl = f.bsize[i - 1];
            const Factor::Blk &fb = f.fwd[i][0];
            // second block of the forward matrix: -S_i^{-1} Lo_i
            gd.push_back({b, bl, b, 0, 0, f.mat.p + fb.off, w.lo_ptr(i), f.mat.p + fb.off + b, fb.cols, bl, fb.cols,
                          -1.0, 0.0});
        }
        run_gemms(gd);
    }
    // last blocks: assemble the remaining block-tridiagonal system densely and invert it
    {
        std::vector<std::pair<const double *, std::pair<double *, int>>> jobs;
        std::vector<int> jn;
        std::vector<DBuf<double>> dense(W.size());
        for (size_t g = 0; g < W.size(); ++g) {
            Work &w = W[g];
            Factor &f = *w.f;
            if (f.lu) continue;
            const int N = f.top_n;
            dense[g].alloc((size_t)N * N);
            launch_fill(dense[g].p, (int64_t)N * N, 0.0, st);
            int64_t ro = 0;
            std::vector<int64_t> offs;
            for (int k : f.top_pos) {
                offs.push_back(ro);
                ro += f.bsize[k];
            }
            for (size_t i = 0; i < f.top_pos.size(); ++i) {
                const int k = f.top_pos[i], b = f.bsize[k];
                double *blk = dense[g].p + offs[i] * N + offs[i];
                THM_HIP(hipMemcpy2DAsync(blk, sizeof(double) * N, w.d_ptr(k), sizeof(double) * b, sizeof(double) * b,
                                         b, hipMemcpyDeviceToDevice, st));
                if (i > 0) {
                    const int kl = f.top_pos[i - 1], bl = f.bsize[kl];
                    // T[i][i-1] = Lo (b x bl), T[i-1][i] = Lo^T
                    THM_HIP(hipMemcpy2DAsync(dense[g].p + offs[i] * N + offs[i - 1], sizeof(double) * N,
                                             w.lo_ptr(k), sizeof(double) * bl, sizeof(double) * bl, b,
                                             hipMemcpyDeviceToDevice, st));
                    launch_transpose(w.lo_ptr(k), b, bl, bl, dense[g].p + offs[i - 1] * N + offs[i], N, 1.0, st);
                }
            }
            jobs.push_back({dense[g].p, {f.mat.p + f.top_off, N}});
            jn.push_back(N);
        }
        THM_HIP(hipStreamSynchronize(st));
        invert(jobs, jn);
    }
    for (Work &w : W) {
        Factor &f = *w.f;
        std::vector<RepackDesc> rd;
        auto add = [&](const Factor::Blk &b) {
            RepackDesc d{};
            d.src = f.mat.p + b.off;
            d.rows = b.rows;
            d.cols = b.cols;
            d.ld = b.ld;
            d.nseg = b.nseg;
            d.poff = b.poff;
            int c = 0;
            for (int q = 0; q < b.nseg; ++q) {
                d.seg_col[q] = c;
                d.seg_len[q] = f.bsize[b.seg_layer[q]];
                d.seg_pstart[q] = b.seg_pstart[q];
                c += d.seg_len[q];
            }
            rd.push_back(d);
        };
        for (auto &lev : f.fwd)
            for (auto &b : lev) add(b);
        for (auto &lev : f.bwd)
            for (auto &b : lev) add(b);
        for (auto &b : f.tops) add(b);
        f.matp.alloc(std::max<int64_t>(f.matp_elems, 1));
        f.matp32.alloc(std::max<int64_t>(f.matp_elems, 1));
        launch_repack(rd, f.matp.p, f.matp32.p, st);
        THM_HIP(hipStreamSynchronize(st));
        f.mat.release();
        // apply layouts: K_ii^{-1} transposed per cell, F and F^T
        if (f.n_int > 0) {
            DBuf<double> kt(f.kiinv.n);
            launch_batch_transpose(f.n_cells, f.n_int, f.n_int, f.kiinv.p, kt.p, st);
            THM_HIP(hipMemcpyAsync(f.kiinv.p, kt.p, sizeof(double) * kt.n, hipMemcpyDeviceToDevice, st));
            THM_HIP(hipStreamSynchronize(st));
        }
        f.FT.alloc(f.F.n);
        launch_batch_transpose(f.n_int > 0 ? f.n_cells : 0, f.ne, f.n_int, f.F.p, f.FT.p, st);
        f.kiinv32.alloc(f.kiinv.n);
        f.F32.alloc(f.F.n);
        f.FT32.alloc(f.F.n);
        launch_convert(f.kiinv.p, f.kiinv32.p, f.kiinv.n, st);
        launch_convert(f.F.p, f.F32.p, f.F.n, st);
        launch_convert(f.FT.p, f.FT32.p, f.FT.n, st);
        w.D.release();
        w.Lo0.release();
        w.lo.clear();
    }
    int32_t hs = 0;
    THM_HIP(hipMemcpyAsync(&hs, status.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    THM_HIP(hipStreamSynchronize(st));
    if (hs) {
        for (thm_system *s : need) s->fac.reset();
        fail(THM_ESINGULAR, "zero or non-finite pivot while factorising the block preconditioner");
    }
    const double dt = now_ms() - t0;
    for (auto &f : facs) {
        f->setup_ms = dt;
        f->bytes = 12 * (f->matp_elems + (int64_t)f->kiinv.n + 2 * (int64_t)f->F.n);
    }
}

}  // namespace thm
