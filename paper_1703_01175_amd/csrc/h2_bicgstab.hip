// BiCGStab (van der Vorst) around the H^2 product, on the device in FP64: the
// iterative solver the paper itself uses for its VIE systems (Sec. V).
//
// x0 = 0, shadow residual r^ = r0 = b.  Each step:
//   rho = <r^, r>;  p = r + (rho / rho_prev)(alpha / omega)(p - omega v)   (p = r first)
//   v = Z p;  alpha = rho / <r^, v>;  s = r - alpha v      (stop when ||s|| / ||b|| <= tol: x += alpha p)
//   t = Z s;  omega = <t, s> / <t, t>;  x += alpha p + omega s;  r = s - omega t
// until ||r|| / ||b|| <= tol; the true residual b - Z x is formed at the end.
// <a, b> = sum conj(a) b.  Reductions are deterministic (fixed-order partial
// sums per group, then one ordered pass).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <mutex>

#include "h2_api_internal.h"

namespace h2 {
namespace {

constexpr int kBlocks = 512;   // partial sums per reduction

using cplx = std::complex<double>;

__device__ __forceinline__ double bsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// part[blk] = this group's share of sum conj(a) b  (re, im)
__global__ __launch_bounds__(256) void kc_dot(const double2* __restrict__ a, const double2* __restrict__ b, int64_t N,
                                              double2* __restrict__ part) {
    __shared__ double red[2][4];
    double sx = 0, sy = 0;
    for (int64_t n = blockIdx.x * 256 + threadIdx.x; n < N; n += int64_t(gridDim.x) * 256) {
        const double2 u = a[n], v = b[n];
        sx += u.x * v.x + u.y * v.y;
        sy += u.x * v.y - u.y * v.x;
    }
    sx = bsum(sx);
    sy = bsum(sy);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = sx;
        red[1][threadIdx.x >> 6] = sy;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        part[blockIdx.x] = make_double2(red[0][0] + red[0][1] + red[0][2] + red[0][3],
                                        red[1][0] + red[1][1] + red[1][2] + red[1][3]);
}

// out[slot] = sum of the partials (one lane, fixed order)
__global__ void kc_finish(const double2* __restrict__ part, int nblk, double2* __restrict__ out, int slot) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double2 s = make_double2(0, 0);
    for (int b = 0; b < nblk; ++b) { s.x += part[b].x; s.y += part[b].y; }
    out[slot] = s;
}

// out = a + c1 b (+ c2 c); optional per-group partial squared norms of out (in part[].x)
__global__ __launch_bounds__(256) void kc_lincomb(const double2* __restrict__ a, const double2* b, double2 c1,
                                                  const double2* __restrict__ c, double2 c2, double2* out, int64_t N,
                                                  double2* __restrict__ part) {
    __shared__ double red[4];
    double nn = 0;
    for (int64_t n = blockIdx.x * 256 + threadIdx.x; n < N; n += int64_t(gridDim.x) * 256) {
        double2 r = a[n];
        const double2 bv = b[n];
        r.x += c1.x * bv.x - c1.y * bv.y;
        r.y += c1.x * bv.y + c1.y * bv.x;
        if (c) {
            const double2 cv = c[n];
            r.x += c2.x * cv.x - c2.y * cv.y;
            r.y += c2.x * cv.y + c2.y * cv.x;
        }
        out[n] = r;
        nn += r.x * r.x + r.y * r.y;
    }
    if (part) {
        nn = bsum(nn);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
        __syncthreads();
        if (threadIdx.x == 0) part[blockIdx.x] = make_double2(red[0] + red[1] + red[2] + red[3], 0.0);
    }
}

struct BiWork {
    double2 *rh, *r, *p, *v, *s, *t, *z, *part, *sc;
};

size_t bi_align(size_t b) { return (b + 255) & ~size_t(255); }

size_t bi_layout(int64_t N, BiWork* W, char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += bi_align(bytes);
        return (double2*)p;
    };
    BiWork w{};
    w.rh = take(N * 16);
    w.r = take(N * 16);
    w.p = take(N * 16);
    w.v = take(N * 16);
    w.s = take(N * 16);
    w.t = take(N * 16);
    w.z = take(N * 16);
    w.part = take(kBlocks * 16);
    w.sc = take(16 * 16);
    if (W) *W = w;
    return off + 256;
}

struct BiSolver {
    const DevH2* d;
    const LevelLaunch* lv;
    hipStream_t s;
    int64_t N;
    int nblk;
    BiWork W;
    double2* host = nullptr;   // 16 complex of host memory

    hipError_t dot(const double2* a, const double2* b, int slot) {
        kc_dot<<<nblk, 256, 0, s>>>(a, b, N, W.part);
        kc_finish<<<1, 64, 0, s>>>(W.part, nblk, W.sc, slot);
        return hipGetLastError();
    }
    // out = a + c1 b + c2 c, its squared norm into sc[slot].x when slot >= 0
    hipError_t lincomb(const double2* a, const double2* b, cplx c1, const double2* c, cplx c2, double2* out, int slot) {
        kc_lincomb<<<nblk, 256, 0, s>>>(a, b, make_double2(c1.real(), c1.imag()), c, make_double2(c2.real(), c2.imag()),
                                        out, N, slot >= 0 ? W.part : nullptr);
        if (slot >= 0) kc_finish<<<1, 64, 0, s>>>(W.part, nblk, W.sc, slot);
        return hipGetLastError();
    }
    hipError_t fetch(int count) {
        hipError_t e = hipMemcpyAsync(host, W.sc, size_t(count) * 16, hipMemcpyDeviceToHost, s);
        return e == hipSuccess ? hipStreamSynchronize(s) : e;
    }
    cplx val(int slot) const { return cplx(host[slot].x, host[slot].y); }
};

}  // namespace
}  // namespace h2

using namespace h2;

extern "C" h2_status h2_bicgstab_workspace(h2_handle h, size_t* bytes) {
    if (!handle_live(h)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (!bytes) return handle_fail(H2_ERR_INVALID_ARG, "null argument");
    *bytes = bi_layout(int64_t(h->dev.n_vox) * kNcomp, nullptr, nullptr);
    return H2_OK;
}

namespace {

h2_status check_args(h2_handle h, const void* b, void* x, double tol, int32_t max_matvec, h2_gmres_report* rep) {
    if (!handle_live(h)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (!b || !x || !rep) return handle_fail(H2_ERR_INVALID_ARG, "null argument");
    if (!(tol > 0.0) || max_matvec < 1) return handle_fail(H2_ERR_INVALID_ARG, "tol must be > 0 and max_matvec >= 1");
    if ((reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(x)) % 16)
        return handle_fail(H2_ERR_INVALID_ARG, "b and x must be 16-byte aligned");
    return H2_OK;
}

// The solve on a workspace at `base` (256-byte aligned, bi_layout bytes); `host`:
// 16 complex of host memory for the scalars read back each step.  Allocates nothing.
h2_status bicgstab_run(h2_handle h, const void* b, void* x, double tol, int32_t max_matvec, h2_gmres_report* rep,
                       char* base, double2* host, hipStream_t stream) {
    const int64_t N = int64_t(h->dev.n_vox) * kNcomp;
    BiSolver S{};
    S.d = &h->dev;
    S.lv = &h->lv;
    S.s = stream;
    S.N = N;
    S.nblk = int(std::min<int64_t>(kBlocks, (N + 255) / 256));
    bi_layout(N, &S.W, base);
    S.host = host;
    *rep = h2_gmres_report{};
    const double2* B = (const double2*)b;
    double2* X = (double2*)x;
    const double2* nul = nullptr;
    int mv = 0, its = 0;
    auto run = [&]() -> h2_status {
        hipError_t e;
        auto dev = [&](hipError_t ee) { return handle_fail(H2_ERR_DEVICE, hipGetErrorString(ee)); };
        // x = 0, r = r^ = b, ||b||
        if ((e = S.lincomb(B, B, cplx(-1, 0), nul, cplx(0, 0), X, -1)) != hipSuccess) return dev(e);
        if ((e = S.lincomb(B, B, cplx(0, 0), nul, cplx(0, 0), S.W.r, 0)) != hipSuccess) return dev(e);
        if ((e = hipMemcpyAsync(S.W.rh, B, N * 16, hipMemcpyDeviceToDevice, S.s)) != hipSuccess) return dev(e);
        if ((e = S.fetch(1)) != hipSuccess) return dev(e);
        const double bnorm = std::sqrt(S.host[0].x);
        if (!std::isfinite(bnorm)) return handle_fail(H2_ERR_NUMERIC, "right-hand side holds NaN or Inf");
        if (bnorm == 0.0) {
            rep->converged = 1;
            return H2_OK;
        }
        cplx rho(1, 0), alpha(1, 0), omega(1, 0);
        double rel = 1.0;
        bool done = false;
        while (mv < max_matvec && !done) {
            if ((e = S.dot(S.W.rh, S.W.r, 1)) != hipSuccess || (e = S.fetch(2)) != hipSuccess) return dev(e);
            const cplx rho_new = S.val(1);
            if (rho_new == cplx(0, 0)) break;                  // breakdown: stop with the current iterate
            if (its == 0) {
                e = S.lincomb(S.W.r, S.W.r, cplx(0, 0), nul, cplx(0, 0), S.W.p, -1);                // p = r
            } else {
                const cplx beta = (rho_new / rho) * (alpha / omega);
                e = S.lincomb(S.W.r, S.W.p, beta, S.W.v, -beta * omega, S.W.p, -1);                // p = r + beta (p - omega v)
            }
            if (e != hipSuccess) return dev(e);
            rho = rho_new;
            if ((e = launch_matvec(*S.d, *S.lv, 1, 0, S.W.p, S.W.v, 1, N, S.s)) != hipSuccess) return dev(e);
            ++mv;
            if ((e = S.dot(S.W.rh, S.W.v, 2)) != hipSuccess || (e = S.fetch(3)) != hipSuccess) return dev(e);
            alpha = rho / S.val(2);
            if ((e = S.lincomb(S.W.r, S.W.v, -alpha, nul, cplx(0, 0), S.W.s, 3)) != hipSuccess ||    // s = r - alpha v
                (e = S.fetch(4)) != hipSuccess)
                return dev(e);
            ++its;
            const double snorm = std::sqrt(S.host[3].x) / bnorm;
            if (!std::isfinite(snorm)) return handle_fail(H2_ERR_NUMERIC, "residual is NaN or Inf");
            if (snorm <= tol) {                                  // x += alpha p, r = s
                if ((e = S.lincomb(X, S.W.p, alpha, nul, cplx(0, 0), X, -1)) != hipSuccess) return dev(e);
                rel = snorm;
                break;
            }
            if ((e = launch_matvec(*S.d, *S.lv, 1, 0, S.W.s, S.W.t, 1, N, S.s)) != hipSuccess) return dev(e);
            ++mv;
            if ((e = S.dot(S.W.t, S.W.s, 4)) != hipSuccess || (e = S.dot(S.W.t, S.W.t, 5)) != hipSuccess ||
                (e = S.fetch(6)) != hipSuccess)
                return dev(e);
            omega = S.val(4) / S.val(5);
            if ((e = S.lincomb(X, S.W.p, alpha, S.W.s, omega, X, -1)) != hipSuccess) return dev(e);   // x += alpha p + omega s
            if ((e = S.lincomb(S.W.s, S.W.t, -omega, nul, cplx(0, 0), S.W.r, 6)) != hipSuccess ||      // r = s - omega t
                (e = S.fetch(7)) != hipSuccess)
                return dev(e);
            rel = std::sqrt(S.host[6].x) / bnorm;
            if (!std::isfinite(rel)) return handle_fail(H2_ERR_NUMERIC, "residual is NaN or Inf");
            done = rel <= tol || omega == cplx(0, 0);
        }
        // true residual b - Z x
        if ((e = launch_matvec(*S.d, *S.lv, 1, 0, X, S.W.z, 1, N, S.s)) != hipSuccess) return dev(e);
        ++mv;
        if ((e = S.lincomb(B, S.W.z, cplx(-1, 0), nul, cplx(0, 0), S.W.z, 7)) != hipSuccess ||
            (e = S.fetch(8)) != hipSuccess)
            return dev(e);
        rel = std::sqrt(S.host[7].x) / bnorm;
        rep->rel_residual = rel;
        rep->converged = rel <= tol;
        return H2_OK;
    };
    h2_status st = run();
    rep->iterations = its;
    rep->matvecs = mv;
    if (hipStreamSynchronize(S.s) != hipSuccess && st >= 0) st = handle_fail(H2_ERR_DEVICE, "solve synchronisation failed");
    if (st < 0) return st;
    return rep->converged ? H2_OK : H2_NOT_CONVERGED;
}

}  // namespace

extern "C" h2_status h2_bicgstab_solve(h2_handle h, const void* b, void* x, double tol, int32_t max_matvec,
                                       h2_gmres_report* rep, void* work, size_t work_bytes, void* stream) {
    h2_status st = check_args(h, b, x, tol, max_matvec, rep);
    if (st != H2_OK) return st;
    if (!work) return handle_fail(H2_ERR_INVALID_ARG, "null argument");
    const int64_t N = int64_t(h->dev.n_vox) * kNcomp;
    if (work_bytes < bi_layout(N, nullptr, nullptr)) return handle_fail(H2_ERR_OOM, "BiCGStab workspace too small");
    char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(work) + 255) & ~uintptr_t(255));
    double2 host[16];                    // scalars read back each step
    return bicgstab_run(h, b, x, tol, max_matvec, rep, base, host, reinterpret_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------- without allocation
// The workspace of h2_bicgstab_solve_static lives in this file-scope device array
// (one copy per device, held until the process ends).  Host code never uses the
// array's name as a device address: the address comes from hipGetSymbolAddress,
// taken once per device with that device current.
namespace {
constexpr size_t kStaticWorkBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) char scratch[kStaticWorkBytes];

namespace {
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (which must be current).
h2_status static_workspace(int dev, char** out) {
    if (dev < 0 || dev >= kMaxDevices) return handle_fail(H2_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return handle_fail(H2_ERR_DEVICE, "static workspace address not available");
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return H2_OK;
}
}  // namespace

extern "C" size_t h2_bicgstab_static_bytes(void) { return kStaticWorkBytes; }

extern "C" h2_status h2_bicgstab_solve_static(h2_handle h, const void* b, void* x, double tol, int32_t max_matvec,
                                              h2_gmres_report* rep, void* stream) {
    h2_status st = check_args(h, b, x, tol, max_matvec, rep);
    if (st != H2_OK) return st;
    const int64_t N = int64_t(h->dev.n_vox) * kNcomp;
    const size_t need = bi_layout(N, nullptr, nullptr);
    if (need > kStaticWorkBytes)
        return handle_fail(H2_ERR_INVALID_ARG, "N too large for the static BiCGStab workspace (needs more than 128 MiB)");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != h->device)
        return handle_fail(H2_ERR_INVALID_ARG, "the handle's device must be current");
    char* base = nullptr;
    if ((st = static_workspace(cur, &base)) != H2_OK) return st;
    double2 host[16];                    // scalars read back each step (pageable host memory)
    return bicgstab_run(h, b, x, tol, max_matvec, rep, base, host, reinterpret_cast<hipStream_t>(stream));
}
