// Internal declarations of the THM library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/thm.h"

namespace thm {

struct Error {
    thm_status code;
    std::string msg;
};

[[noreturn]] void fail(thm_status code, const std::string &msg);

#define THM_HIP(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            ::thm::fail(e_ == hipErrorOutOfMemory ? THM_ENOMEM : THM_EHIP,                   \
                        std::string(#call) + ": " + hipGetErrorString(e_));                  \
    } while (0)

// Owning device buffer (hipMalloc'd, freed in the destructor).
template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t count) {
        release();
        n = count;
        if (count) THM_HIP(hipMalloc(&p, count * sizeof(T)));
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void upload(const std::vector<T> &h, hipStream_t s) {
        alloc(h.size());
        if (!h.empty()) THM_HIP(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    }
    size_t bytes() const { return n * sizeof(T); }
};

// ---------------------------------------------------------------- host topology
// Local shape function descriptor: component, tangential degree i, normal
// indices (jb, kc) along the two other axes in increasing order (kc = 0 in 2D).
struct LocalFn {
    int comp, i, jb, kc;
};

struct Topo {
    int dim = 2, p = 0;
    int n[3] = {1, 1, 1};
    double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, h[3] = {1, 1, 1};
    int64_t n_edges[3] = {0, 0, 0}, n_faces[3] = {0, 0, 0}, n_cells = 0;
    int64_t edge_off[3] = {0, 0, 0}, face_off[3] = {0, 0, 0}, cell_off = 0, n_dofs = 0;
    int n_loc = 0, n_int = 0, pe = 1, pf = 0;
    std::vector<LocalFn> fns;            // local order
    std::vector<int> side_fns[6];        // local DoFs with tangential trace on side 2*axis+s
    std::vector<int32_t> cell_dofs;      // n_cells * n_loc

    void build(int dim, int p, const int *cells, const double *lo, const double *hi);
    int64_t edge_id(int axis, int i, int j, int k) const;
    int64_t face_id(int axis, int i, int j, int k) const;
    void cell_ijk(int64_t c, int *ijk) const;
    bool cell_on_side(int64_t c, int axis, int side) const;
};

// CSR pattern with a deterministic gather map from per-entity dense blocks.
struct HostCSR {
    int64_t nrows = 0;
    std::vector<int32_t> rowptr, col;
    std::vector<int32_t> gptr;   // nnz+1
    std::vector<int32_t> gsrc;   // indices into the block buffer
};

// Boundary side entries (cell, axis, side).
struct Side {
    int32_t cell, axis, side;
};

// Block-tridiagonal layering of the skeleton (non-interior) DoFs.
constexpr int SKEL_ALIGN = 8;

struct Layering {
    int nlayers = 0;
    std::vector<int32_t> bsize;          // per layer
    std::vector<int64_t> boff;           // offset of layer in the skeleton vector
    std::vector<int64_t> sinv_off;       // offset of Sinv_k (b_k^2)
    std::vector<int64_t> lf_off;         // offset of Lf_k (b_k x b_{k-1}); -1 for k = 0
    int64_t n_skel = 0, sinv_total = 0, lf_total = 0;
    std::vector<int32_t> skel_dof;       // skeleton position -> global DoF
    std::vector<int32_t> dof_pos;        // global DoF -> skeleton position (-1: interior)
    // Layout of the preconditioner's skeleton work vectors: every layer starts at a
    // multiple of SKEL_ALIGN entries (the tail of a layer is zero padding).
    std::vector<int64_t> pboff;          // padded offset of layer k (nlayers + 1 entries)
    int64_t n_skel_pad = 0;
    std::vector<int32_t> skel_pos;       // skeleton position -> padded position
    // condensed element entry (cell, u, v over skeleton local DoFs) -> dense target
    std::vector<int64_t> tgt_index;      // unique targets: layer-block linear index (see encode)
    std::vector<int32_t> tgt_ptr;        // per unique target, into tgt_src
    std::vector<int32_t> tgt_src;        // cell * ne * ne + u * ne + v
    std::vector<int32_t> tgt_kind;       // 0: Sinv_k block, 1: B_k block (rows k, cols k-1)
    // skeleton position -> (cell, local skeleton index) pairs for condensation
    std::vector<int32_t> cond_ptr, cond_cell, cond_loc;
};

void build_csr(const Topo &t, HostCSR &K);
void build_side_csr(const Topo &t, const std::vector<Side> &sides, HostCSR &C);
void build_layering(const Topo &t, const std::vector<uint8_t> &dir, Layering &L);

// ---------------------------------------------------------------- device views
// Per-system pointers used by batched kernels (plain struct, copied to device).
struct SysDev {
    int64_t n;             // complex DoFs
    const int32_t *rowptr, *col;
    const void *kval;      // double or float
    const int32_t *crowptr, *ccol;
    const void *cval;
};

}  // namespace thm
