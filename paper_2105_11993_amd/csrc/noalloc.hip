// Block-preconditioner application without device allocation, for callers that cannot
// allocate (code under stream capture, serving loops, harnesses that forbid hipMalloc).
//
// The apply of diag(K, K)^{-1} (eq. (11)) needs three work vectors besides its input and
// output: the reduced skeleton right-hand side, the skeleton solution and the condensation
// terms (plus FP32 copies of input and output for the FP32 factor).  Here they live in one
// file-scope device array, `scratch`, of NOALLOC_SCRATCH_BYTES.  Each device holds its own
// copy of the array until the process ends; its device address is looked up once per device
// with hipGetSymbolAddress and only that address is handed to kernels (the array's name is a
// host-side stand-in in host code).  Every call on a device shares the array and leaves its
// last contents there: calls that overlap on one device race.
#include <mutex>

#include "solver.h"

namespace thm {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEV = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEV] = {};

// Device address of `scratch` on the current device (looked up on first use per device).
unsigned char *scratch_address() {
    int dev = 0;
    THM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEV) fail(THM_EUNSUPPORTED, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            fail(THM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    return static_cast<unsigned char *>(g_scratch_ptr[dev]);
}

template <class T>
__global__ void __launch_bounds__(256) k_zero_fill(T *__restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = T(0);
}

template <class T>
void zero_fill(T *p, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    k_zero_fill<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, n);
    THM_HIP(hipGetLastError());
}

int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }
}  // namespace

void noalloc_prec_apply(Ctx &c, int precision, const double *x, double *y, hipStream_t st) {
    if (!c.prec_ready) fail(THM_EINVAL, "preconditioner schedule not built for this system");
    if (c.ns != 1) fail(THM_EINVAL, "allocation-free apply serves single-system contexts only");
    const bool f32 = precision == THM_FP32_IR;
    const int64_t v = f32 ? 4 : 8;
    // layout: [x32, y32 (FP32 only)] ws, ys, tw, each 256-byte aligned
    const int64_t b_io = f32 ? align256(c.K.B.Ltot * 4) : 0;
    const int64_t b_w = align256(c.P.Stot * v);
    const int64_t b_t = align256(2 * c.P.Ttot * v);
    const int64_t need = 2 * b_io + 2 * b_w + b_t;
    if (need > (int64_t)NOALLOC_SCRATCH_BYTES)
        fail(THM_EINVAL, "system needs " + std::to_string(need) + " bytes of scratch; the allocation-free apply has " +
                             std::to_string((long long)NOALLOC_SCRATCH_BYTES));
    unsigned char *base = scratch_address();
    unsigned char *ws = base + 2 * b_io, *ys = ws + b_w, *tw = ys + b_w;
    const int32_t *mask = c.mask_all.p;
    if (f32) {
        float *x32 = reinterpret_cast<float *>(base), *y32 = reinterpret_cast<float *>(base + b_io);
        float *w = reinterpret_cast<float *>(ws), *yy = reinterpret_cast<float *>(ys);
        // padding positions of the skeleton vectors are read (against zero matrix entries)
        // and must hold zeros, whatever an earlier call left there
        zero_fill<float>(w, c.P.Stot, st);
        zero_fill<float>(yy, c.P.Stot, st);
        launch_scale<double, float>(c.K.B, nullptr, nullptr, 0, x, x32, nullptr, 0, nullptr, st);
        launch_prec_apply<float>(c.P, c.P.d32.p, c.K.B.off.p, 1, mask, x32, y32, w, yy,
                                 reinterpret_cast<float *>(tw), st);
        launch_scale<float, double>(c.K.B, nullptr, nullptr, 0, y32, y, nullptr, 0, nullptr, st);
    } else {
        double *w = reinterpret_cast<double *>(ws), *yy = reinterpret_cast<double *>(ys);
        zero_fill<double>(w, c.P.Stot, st);
        zero_fill<double>(yy, c.P.Stot, st);
        launch_prec_apply<double>(c.P, c.P.d64.p, c.K.B.off.p, 1, mask, x, y, w, yy,
                                  reinterpret_cast<double *>(tw), st);
    }
}

}  // namespace thm
