// Restarted GMRES(m) around the H^2 product, on the device in FP64.
//
// The paper solves its VIE system iteratively with the O(N) H^2 product inside
// the iteration (Sec. IV.B, Sec. V).  Each Arnoldi step here is
//   w = Z v_j;  h = V^H w, w -= V h  (classical Gram-Schmidt), and when that
//   left less than 1/sqrt(2) of ||w|| a second pass h' = V^H w, w -= V h',
//   h += h' (the Daniel-Gragg-Kaufman-Stewart test);  v_{j+1} = w / ||w||;
//   Givens update of the Hessenberg column and of the residual estimate |g_{j+1}|.
// A cycle ends at m steps, on breakdown, or when the estimate reaches the
// tolerance; then y = R^-1 g, x += V y, and the true residual b - Z x decides.
// The second-pass test and the stopping test are taken on the device (per-solve
// flags gate the kernels of later steps), and the host reads each step's record
// one step late: it has already queued the next step, so the device never waits
// for the host inside a cycle.  A step queued after the one that ended the cycle
// does no Arnoldi work; only its product is spent.
// With a lower-precision product the solve is iterative refinement: an FP64
// outer residual and an inner GMRES (FP64 Arnoldi) on the FP32 / BF16 blocks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "h2_api_internal.h"
#include "h2_givens.h"

namespace h2 {
namespace {

constexpr int kDotTile = 16;      // basis vectors per dot-product pass
constexpr double kDgks = 0.70710678118654752;   // repeat Gram-Schmidt when the norm drops below this fraction
constexpr int kDotBlocks = 512;   // partial sums per vector

__device__ __forceinline__ double2 cmul_conj(double2 a, double2 b) {   // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

template <int W>
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v += __shfl_down(v, o, W);
    return v;
}

// Per-solve device flags: [0] the cycle has stopped (set by k_givens_step), [1] this
// step needs the second Gram-Schmidt pass, [2] steps that took it.  A kernel given
// flags runs only while the cycle goes on (and, for the second pass, when needed).
__device__ __forceinline__ bool gate_open(const int* flags, int second) {
    return !flags || (flags[0] == 0 && (!second || flags[1] != 0));
}

// partial[blk][i] = sum over this block's elements of conj(V_i[n]) w[n], i in [i0, i0 + 16);
// with nrm_partial, the y = 0 blocks also leave their share of ||w||^2 there
__global__ __launch_bounds__(256) void k_multidot(const double2* __restrict__ V, int64_t ldv, int nvec,
                                                  const double2* __restrict__ w, int64_t N,
                                                  double2* __restrict__ partial, double* __restrict__ nrm_partial,
                                                  const int* __restrict__ flags, int second) {
    if (!gate_open(flags, second)) return;
    __shared__ double2 red[4][kDotTile];
    __shared__ double nred[4];
    const int i0 = blockIdx.y * kDotTile;
    const int cnt = min(kDotTile, nvec - i0);
    const bool with_norm = nrm_partial && blockIdx.y == 0;
    double2 acc[kDotTile];
    double nn = 0;
#pragma unroll
    for (int q = 0; q < kDotTile; ++q) acc[q] = make_double2(0, 0);
    for (int64_t n = blockIdx.x * 256 + threadIdx.x; n < N; n += int64_t(gridDim.x) * 256) {
        const double2 wv = w[n];
        nn += wv.x * wv.x + wv.y * wv.y;
#pragma unroll
        for (int q = 0; q < kDotTile; ++q)
            if (q < cnt) {
                double2 p = cmul_conj(V[(int64_t)(i0 + q) * ldv + n], wv);
                acc[q].x += p.x;
                acc[q].y += p.y;
            }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kDotTile; ++q) {
        double rx = wave_sum<64>(acc[q].x);
        double ry = wave_sum<64>(acc[q].y);
        if (lane == 0) red[wv][q] = make_double2(rx, ry);
    }
    if (with_norm) {
        nn = wave_sum<64>(nn);
        if (lane == 0) nred[wv] = nn;
    }
    __syncthreads();
    if (threadIdx.x < cnt) {
        const int q = threadIdx.x;
        double2 s = red[0][q];
        for (int k = 1; k < 4; ++k) { s.x += red[k][q].x; s.y += red[k][q].y; }
        partial[(int64_t)blockIdx.x * 128 + i0 + q] = s;
    }
    if (with_norm && threadIdx.x == 0) nrm_partial[blockIdx.x] = nred[0] + nred[1] + nred[2] + nred[3];
}

// Block i < nvec: out[i] (+)= sum over blk of partial[blk][i]; block nvec (when
// nrm_partial): scal[nrm_slot] = sqrt(sum of nrm_partial).  Fixed summation order.
__global__ __launch_bounds__(256) void k_reduce_dots(const double2* __restrict__ partial, int nblk, int nvec,
                                                     double2* __restrict__ out, int accumulate,
                                                     const double* __restrict__ nrm_partial, double* __restrict__ scal,
                                                     int nrm_slot, const int* __restrict__ flags, int second) {
    if (!gate_open(flags, second)) return;
    __shared__ double red[2][4];
    const int i = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double sx = 0, sy = 0;
    if (i < nvec) {
        for (int b = threadIdx.x; b < nblk; b += 256) {
            const double2 p = partial[(int64_t)b * 128 + i];
            sx += p.x;
            sy += p.y;
        }
    } else {
        for (int b = threadIdx.x; b < nblk; b += 256) sx += nrm_partial[b];
    }
    sx = wave_sum<64>(sx);
    sy = wave_sum<64>(sy);
    if (lane == 0) {
        red[0][wv] = sx;
        red[1][wv] = sy;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    sx = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    sy = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    if (i < nvec) {
        if (accumulate) { sx += out[i].x; sy += out[i].y; }
        out[i] = make_double2(sx, sy);
    } else {
        scal[nrm_slot] = sqrt(sx);
    }
}


// w[n] += sign * sum_i V_i[n] c_i  (sign = -1: orthogonalise; +1: x += V y)
// optional: partial squared norms of the result (nrm_partial[blockIdx.x])
__global__ __launch_bounds__(256) void k_multiaxpy(const double2* __restrict__ V, int64_t ldv, int nvec,
                                                   const double2* __restrict__ c, double sign, double2* __restrict__ w,
                                                   int64_t N, double* __restrict__ nrm_partial,
                                                   const int* __restrict__ flags = nullptr, int second = 0) {
    if (!gate_open(flags, second)) return;
    __shared__ double2 cs[128];
    __shared__ double red[4];
    for (int i = threadIdx.x; i < nvec; i += 256) cs[i] = c[i];
    __syncthreads();
    double nn = 0;
    for (int64_t n = blockIdx.x * 256 + threadIdx.x; n < N; n += int64_t(gridDim.x) * 256) {
        double2 a = make_double2(0, 0);
        for (int i = 0; i < nvec; ++i) {
            const double2 v = V[(int64_t)i * ldv + n];
            const double2 ci = cs[i];
            a.x = fma(v.x, ci.x, a.x);
            a.x = fma(-v.y, ci.y, a.x);
            a.y = fma(v.x, ci.y, a.y);
            a.y = fma(v.y, ci.x, a.y);
        }
        double2 r = w[n];
        r.x += sign * a.x;
        r.y += sign * a.y;
        w[n] = r;
        nn += r.x * r.x + r.y * r.y;
    }
    if (nrm_partial) {
        nn = wave_sum<64>(nn);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
        __syncthreads();
        if (threadIdx.x == 0) nrm_partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

// r = b - z, partial squared norms
__global__ __launch_bounds__(256) void k_residual(const double2* __restrict__ b, const double2* __restrict__ z,
                                                  double2* __restrict__ r, int64_t N, double* __restrict__ nrm_partial) {
    __shared__ double red[4];
    double nn = 0;
    for (int64_t n = blockIdx.x * 256 + threadIdx.x; n < N; n += int64_t(gridDim.x) * 256) {
        double2 v = make_double2(b[n].x - z[n].x, b[n].y - z[n].y);
        r[n] = v;
        nn += v.x * v.x + v.y * v.y;
    }
    nn = wave_sum<64>(nn);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
    __syncthreads();
    if (threadIdx.x == 0) nrm_partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// partial squared norms of a vector
__global__ __launch_bounds__(256) void k_norm2(const double2* __restrict__ a, int64_t N, double* __restrict__ nrm_partial) {
    __shared__ double red[4];
    double nn = 0;
    for (int64_t n = blockIdx.x * 256 + threadIdx.x; n < N; n += int64_t(gridDim.x) * 256) {
        double2 v = a[n];
        nn += v.x * v.x + v.y * v.y;
    }
    nn = wave_sum<64>(nn);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
    __syncthreads();
    if (threadIdx.x == 0) nrm_partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// sum of partial norms -> scal[slot] = sqrt(sum)  (one wave, fixed order)
__global__ void k_finish_norm(const double* __restrict__ partial, int nblk, double* __restrict__ scal, int slot) {
    double s = 0;
    for (int b = threadIdx.x; b < nblk; b += 64) s += partial[b];
    s = wave_sum<64>(s);
    if (threadIdx.x == 0) scal[slot] = sqrt(s);
}

// After a Gram-Schmidt pass: scal[0] = ||w|| from the partial norms.  First pass
// (second = 0): flags[1] = the second pass is needed (||w|| below 1/sqrt(2) of the
// norm before, scal[5], or not a number).  Second pass: runs only when needed.
__global__ void k_finish_pass(const double* __restrict__ partial, int nblk, double* __restrict__ scal,
                              int* __restrict__ flags, int second) {
    if (!gate_open(flags, second)) return;
    double s = 0;
    for (int b = threadIdx.x; b < nblk; b += 64) s += partial[b];
    s = wave_sum<64>(s);
    if (threadIdx.x == 0) {
        const double nw = sqrt(s);
        scal[0] = nw;
        if (!second) flags[1] = !(nw >= kDgks * scal[5]);
    }
}

// dst = src * (1 / scal[slot])
__global__ void k_scale(const double2* __restrict__ src, double2* __restrict__ dst, int64_t N,
                        const double* __restrict__ scal, int slot, const int* __restrict__ flags = nullptr) {
    if (!gate_open(flags, 0)) return;
    const double inv = 1.0 / scal[slot];
    for (int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; n < N; n += int64_t(gridDim.x) * blockDim.x)
        dst[n] = make_double2(src[n].x * inv, src[n].y * inv);
}

__global__ void k_fill(double2* __restrict__ a, int64_t N) {
    for (int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; n < N; n += int64_t(gridDim.x) * blockDim.x)
        a[n] = make_double2(0, 0);
}

__global__ void k_add(double2* __restrict__ x, const double2* __restrict__ d, int64_t N) {
    for (int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; n < N; n += int64_t(gridDim.x) * blockDim.x) {
        x[n].x += d[n].x;
        x[n].y += d[n].y;
    }
}



// One Arnoldi step's Givens update of Hessenberg column j and its stopping test, on the device:
// the cycle stops on breakdown (||w|| = 0), when |g_{j+1}| / ||b|| (scal[2]) reaches
// tol, or on a value that is not a number.  rec = {||w||, |g_{j+1}|, stop} for the
// host; flags[2] counts the steps that took a second Gram-Schmidt pass.
__global__ void k_givens_step(double2* __restrict__ H, int ldh, int j, const double2* __restrict__ hcol,
                              double* __restrict__ cs, double2* __restrict__ sn, double2* __restrict__ g,
                              double* __restrict__ scal, int* __restrict__ flags, double tol, double* __restrict__ rec) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || flags[0] != 0) return;
    double2* col = H + (int64_t)j * ldh;
    for (int i = 0; i <= j; ++i) col[i] = hcol[i];
    col[j + 1] = make_double2(scal[0], 0.0);
    const double est = givens_column(col, j, cs, sn, g);
    scal[1] = est;
    const double hn = scal[0];
    const bool stop = hn == 0.0 || !(est / scal[2] > tol) || !isfinite(hn) || !isfinite(est);
    flags[2] += flags[1];
    flags[0] = stop ? 1 : 0;
    rec[0] = hn;
    rec[1] = est;
    rec[2] = stop ? 1.0 : 0.0;
}

// Minimal-residual step of the restart correction: alpha = w^H r / ||w||^2 from the dot
// (hc[0]) and the partial norms of w; scal[10..11] = alpha (0 when ||w|| = 0 or alpha is
// not a number).
__global__ void k_mr_alpha(const double* __restrict__ partial, int nblk, const double2* __restrict__ hc,
                           double* __restrict__ scal) {
    double s = 0;
    for (int b = threadIdx.x; b < nblk; b += 64) s += partial[b];
    s = wave_sum<64>(s);
    if (threadIdx.x == 0) {
        double ar = 0.0, ai = 0.0;
        if (s > 0.0) {
            ar = hc[0].x / s;
            ai = hc[0].y / s;
            if (!isfinite(ar) || !isfinite(ai)) ar = ai = 0.0;
        }
        scal[10] = ar;
        scal[11] = ai;
    }
}

// x += alpha c, r -= alpha w (alpha = scal[10..11]); partial squared norms of the new r
__global__ __launch_bounds__(256) void k_mr_step(double2* __restrict__ x, const double2* __restrict__ c,
                                                 double2* __restrict__ r, const double2* __restrict__ w, int64_t N,
                                                 const double* __restrict__ scal, double* __restrict__ nrm_partial) {
    __shared__ double red[4];
    const double ar = scal[10], ai = scal[11];
    double nn = 0;
    for (int64_t n = blockIdx.x * 256 + threadIdx.x; n < N; n += int64_t(gridDim.x) * 256) {
        const double2 cv = c[n], wv = w[n];
        double2 xv = x[n], rv = r[n];
        xv.x += ar * cv.x - ai * cv.y;
        xv.y += ar * cv.y + ai * cv.x;
        rv.x -= ar * wv.x - ai * wv.y;
        rv.y -= ar * wv.y + ai * wv.x;
        x[n] = xv;
        r[n] = rv;
        nn += rv.x * rv.x + rv.y * rv.y;
    }
    nn = wave_sum<64>(nn);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
    __syncthreads();
    if (threadIdx.x == 0) nrm_partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// A new cycle: g = (beta, 0, ..., 0) and the step flags cleared.
__global__ void k_init_cycle(double2* __restrict__ g, int m, const double* __restrict__ scal, int slot,
                             int* __restrict__ flags) {
    for (int i = threadIdx.x; i <= m; i += blockDim.x) g[i] = make_double2(i == 0 ? scal[slot] : 0.0, 0.0);
    if (threadIdx.x == 0) {
        flags[0] = 0;
        flags[1] = 0;
    }
}

// h = h' + h after the second pass (when it ran)
__global__ void k_add_dots(const double2* __restrict__ y, int nvec, double2* __restrict__ h,
                           const int* __restrict__ flags) {
    if (!gate_open(flags, 1)) return;
    const int i = threadIdx.x;
    if (i < nvec) h[i] = make_double2(y[i].x + h[i].x, y[i].y + h[i].y);
}

__global__ void k_zero_flags(int* __restrict__ flags) {
    if (threadIdx.x < 4) flags[threadIdx.x] = 0;
}

// y = R^-1 g on the leading k x k triangle (single thread)
__global__ void k_backsolve(const double2* __restrict__ H, int ldh, int k, const double2* __restrict__ g,
                            double2* __restrict__ y) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    back_substitute(H, ldh, k, g, y);
}


struct Work {
    double2 *V, *Zs, *w, *r, *z, *d, *xs, *hcol, *H, *sn, *g, *y;
    float *mX, *mH1, *mH2, *mY;
    double* mnorm;
    float2 *lo_in, *lo_out;
    double *cs, *scal, *npart;
    int* flags;                    // per-solve step flags (see gate_open)
    double* rec;                   // two step records {||w||, |g|, stop, -} read by the host
    double2* dpart;
    int64_t ldv;
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t work_layout(int64_t N, int m, Work* W, char* base, int precond = 0, int64_t nleaf = 0, int n_in = 0,
                   int n_hidden = 0, int n_out = 0) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    const int64_t ldv = (N + 15) / 16 * 16;
    Work w{};
    w.ldv = ldv;
    w.V = (double2*)take(size_t(ldv) * (m + 1) * 16);
    w.Zs = precond ? (double2*)take(size_t(ldv) * m * 16) : nullptr;
    if (precond >= 2) {
        w.mX = (float*)take(size_t(nleaf) * n_in * 4);
        w.mH1 = (float*)take(size_t(nleaf) * n_hidden * 4);
        w.mH2 = (float*)take(size_t(nleaf) * n_hidden * 4);
        w.mY = (float*)take(size_t(nleaf) * n_out * 4);
        w.mnorm = (double*)take(64);
    }
    w.w = (double2*)take(N * 16);
    w.r = (double2*)take(N * 16);
    w.z = (double2*)take(N * 16);
    w.d = (double2*)take(N * 16);
    w.xs = (double2*)take(N * 16);
    w.lo_in = (float2*)take(N * 8);
    w.lo_out = (float2*)take(N * 8);
    w.hcol = (double2*)take(128 * 16);
    w.H = (double2*)take(size_t(m + 1) * m * 16);
    w.cs = (double*)take(128 * 8);
    w.sn = (double2*)take(128 * 16);
    w.g = (double2*)take(130 * 16);
    w.y = (double2*)take(128 * 16);
    w.scal = (double*)take(64 * 8);
    w.flags = (int*)take(4 * 4);
    w.rec = (double*)take(8 * 8);
    w.npart = (double*)take(kDotBlocks * 8);
    w.dpart = (double2*)take(size_t(kDotBlocks) * 128 * 16);
    if (W) *W = w;
    return off + 256;
}

struct Solver {
    h2_handle h;
    int precond = 0;
    const DevH2* d;
    const LevelLaunch* lv;
    hipStream_t s;
    int64_t N;
    Work W;
    double* host = nullptr;   // pinned host scalars
    int nblk;

    hipError_t matvec(int prec, const double2* x, double2* y) {
        if (prec == 0) return launch_matvec(*d, *lv, 1, 0, x, y, 1, N, s);
        hipError_t e = launch_vec_to_fp32(x, W.lo_in, N, s);
        if (e != hipSuccess) return e;
        if (prec == H2_BF16X3) {   // the batched tier's group holding this handle alone, one column
            const void* xin[1] = {W.lo_in};
            void* yout[1] = {W.lo_out};
            const int64_t nr[1] = {1}, lds[1] = {N};
            if (group_run(h->self_group, 1, xin, yout, nr, lds, s) != H2_OK) return hipErrorLaunchFailure;
        } else {
            e = launch_matvec(*d, *lv, 1, prec, W.lo_in, W.lo_out, 1, N, s);
            if (e != hipSuccess) return e;
        }
        return launch_vec_to_fp64(W.lo_out, y, N, s);
    }

    hipError_t norm_into(const double2* a, int slot) {
        k_norm2<<<nblk, 256, 0, s>>>(a, N, W.npart);
        k_finish_norm<<<1, 64, 0, s>>>(W.npart, nblk, W.scal, slot);
        return hipGetLastError();
    }

    hipError_t fetch(int count) {   // copy scal[0..count) to host and wait
        hipError_t e = hipMemcpyAsync(host, W.scal, count * 8, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(s);
    }

    // V^H w for vectors 0..nvec-1 into out (accumulate or overwrite); with norm_slot >= 0
    // also scal[norm_slot] = ||w||; gated by the step flags (second: the second pass)
    void multidot(int nvec, const double2* w, double2* out, int accumulate, int norm_slot, int second) {
        dim3 grid(nblk, (nvec + kDotTile - 1) / kDotTile);
        double* np = norm_slot >= 0 ? W.npart : nullptr;
        k_multidot<<<grid, 256, 0, s>>>(W.V, W.ldv, nvec, w, N, W.dpart, np, W.flags, second);
        k_reduce_dots<<<nvec + (np ? 1 : 0), 256, 0, s>>>(W.dpart, nblk, nvec, out, accumulate, np, W.scal,
                                                          norm_slot, W.flags, second);
    }
    hipEvent_t ev[2] = {nullptr, nullptr};   // step records copied to host[16 + 4 (j & 1)]

    // Arnoldi's right preconditioner: 0 none, 1 block diagonal, 2 MLP.  With the
    // restart correction (precond 3) the cycles use the MLP's base map.
    int inner_pc() const { return precond == 3 ? (h->mlp_base == H2_PRECOND_BLOCKDIAG ? 1 : 0) : precond; }

    // z = P(v) for the right preconditioner
    hipError_t apply_precond(const double2* v, double2* z) {
        if (inner_pc() == 1) return launch_bd_apply(d->leaves, d->perm, (const double2*)h->bd_buf, v, z, s);
        return mlp_apply_handle(h, v, z, W.mX, W.mH1, W.mH2, W.mY, W.mnorm, s);
    }

    // Learned correction at a cycle start: c = P(r) with the attached MLP map, w = Z c,
    // and the step x += alpha c, r -= alpha w with alpha = w^H r / ||w||^2 (the multiple
    // of c that minimises the residual; none when w = 0).  beta and scal[3] follow r.
    h2_status restart_correction(int prec, double2* x, double* beta, int* mv) {
        hipError_t e;
        if ((e = mlp_apply_handle(h, W.r, W.w, W.mX, W.mH1, W.mH2, W.mY, W.mnorm, s)) != hipSuccess)
            return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
        if ((e = matvec(prec, W.w, W.z)) != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
        ++*mv;
        k_multidot<<<dim3(nblk, 1), 256, 0, s>>>(W.z, W.ldv, 1, W.r, N, W.dpart, nullptr, nullptr, 0);   // w^H r
        k_reduce_dots<<<1, 256, 0, s>>>(W.dpart, nblk, 1, W.hcol, 0, nullptr, W.scal, 0, nullptr, 0);
        k_norm2<<<nblk, 256, 0, s>>>(W.z, N, W.npart);                                             // ||w||^2
        k_mr_alpha<<<1, 64, 0, s>>>(W.npart, nblk, W.hcol, W.scal);
        k_mr_step<<<nblk, 256, 0, s>>>(x, W.w, W.r, W.z, N, W.scal, W.npart);
        k_finish_norm<<<1, 64, 0, s>>>(W.npart, nblk, W.scal, 4);
        if ((e = fetch(12)) != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
        if (host[10] != 0.0 || host[11] != 0.0) {        // a step was taken
            if ((e = hipMemcpyAsync(W.scal + 3, W.scal + 4, 8, hipMemcpyDeviceToDevice, s)) != hipSuccess)
                return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
            *beta = host[4];
            ++corrections;
        }
        return H2_OK;
    }
    int corrections = 0;
    int reorth = 0;                    // Arnoldi steps that repeated Gram-Schmidt

    // GMRES(m) on Z x = rhs from x0 = 0, or from the given x when use_x0 (x overwritten).
    // prec: product tier.  Returns status; fills its/mv/restarts and the final true relative residual.
    h2_status gmres(int prec, const double2* rhs, double2* x, int m, int max_mv, double tol, int* its, int* mv,
                    int* restarts, double* relres, bool use_x0 = false) {
        hipError_t e;
        *its = 0;
        *mv = 0;
        *restarts = 0;
        if (use_x0) {
            // r = rhs - Z x0
            if ((e = matvec(prec, x, W.z)) != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
            ++*mv;
            k_residual<<<nblk, 256, 0, s>>>(rhs, W.z, W.r, N, W.npart);
        } else {
            k_fill<<<nblk, 256, 0, s>>>(x, N);
            e = hipMemcpyAsync(W.r, rhs, N * 16, hipMemcpyDeviceToDevice, s);   // r = rhs (x0 = 0)
            if (e != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
        }
        (void)norm_into(rhs, 2);              // scal[2] = ||b||
        (void)norm_into(W.r, 3);              // scal[3] = ||r||
        if ((e = fetch(4)) != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
        const double bnorm = host[2];
        if (!std::isfinite(bnorm)) return handle_fail(H2_ERR_NUMERIC, "right-hand side holds NaN or Inf");
        if (bnorm == 0.0) {   // Z x = 0 has the unique solution x = 0, whatever x0 was
            k_fill<<<nblk, 256, 0, s>>>(x, N);
            *relres = 0.0;
            return H2_OK;
        }
        double beta = host[3];
        const int ipc = inner_pc();
        while (true) {
            *relres = beta / bnorm;
            if (!std::isfinite(beta)) return handle_fail(H2_ERR_NUMERIC, "residual is NaN or Inf");
            if (*relres <= tol) return H2_OK;
            if (*mv >= max_mv) return H2_NOT_CONVERGED;
            if (precond == 3) {
                h2_status st = restart_correction(prec, x, &beta, mv);
                if (st != H2_OK) return st;
                *relres = beta / bnorm;
                if (*relres <= tol) return H2_OK;
                if (*mv >= max_mv) return H2_NOT_CONVERGED;
            }
            // v_0 = r / beta
            k_scale<<<nblk, 256, 0, s>>>(W.r, W.V, N, W.scal, 3);
            k_init_cycle<<<1, 256, 0, s>>>(W.g, m, W.scal, 3, W.flags);
            int jend = 0, pending = -1;
            for (int j = 0; j <= m; ++j) {
                const bool queue = j < m && *mv < max_mv;
                if (queue) {
                    double2* vj = W.V + (int64_t)j * W.ldv;
                    const double2* zj = vj;
                    if (ipc) {
                        double2* zz = W.Zs + (int64_t)j * W.ldv;
                        if ((e = apply_precond(vj, zz)) != hipSuccess)
                            return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
                        zj = zz;
                    }
                    if ((e = matvec(prec, zj, W.w)) != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
                    ++*mv;
                    // classical Gram-Schmidt with ||w|| before it; repeated when the norm fell below
                    // 1/sqrt(2) of that (the Daniel-Gragg-Kaufman-Stewart test), decided on the device
                    multidot(j + 1, W.w, W.hcol, 0, 5, 0);                                 // h = V^H w, ||w||
                    k_multiaxpy<<<nblk, 256, 0, s>>>(W.V, W.ldv, j + 1, W.hcol, -1.0, W.w, N, W.npart, W.flags, 0);
                    k_finish_pass<<<1, 64, 0, s>>>(W.npart, nblk, W.scal, W.flags, 0);    // ||w - V h||, test
                    multidot(j + 1, W.w, W.y, 0, -1, 1);                                   // h' = V^H w
                    k_multiaxpy<<<nblk, 256, 0, s>>>(W.V, W.ldv, j + 1, W.y, -1.0, W.w, N, W.npart, W.flags, 1);
                    k_add_dots<<<1, 128, 0, s>>>(W.y, j + 1, W.hcol, W.flags);             // h += h'
                    k_finish_pass<<<1, 64, 0, s>>>(W.npart, nblk, W.scal, W.flags, 1);     // ||w||
                    double* rec = W.rec + 4 * (j & 1);
                    k_givens_step<<<1, 1, 0, s>>>(W.H, m + 1, j, W.hcol, W.cs, W.sn, W.g, W.scal, W.flags, tol, rec);
                    k_scale<<<nblk, 256, 0, s>>>(W.w, W.V + (int64_t)(j + 1) * W.ldv, N, W.scal, 0, W.flags);
                    if ((e = hipMemcpyAsync(host + 16 + 4 * (j & 1), rec, 32, hipMemcpyDeviceToHost, s)) != hipSuccess ||
                        (e = hipEventRecord(ev[j & 1], s)) != hipSuccess)
                        return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
                }
                if (pending >= 0) {            // the previous step's record, read while this one runs
                    if ((e = hipEventSynchronize(ev[pending & 1])) != hipSuccess)
                        return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
                    const double* r = host + 16 + 4 * (pending & 1);
                    if (!std::isfinite(r[0]) || !std::isfinite(r[1]))
                        return handle_fail(H2_ERR_NUMERIC, "Arnoldi produced NaN or Inf");
                    jend = pending + 1;
                    ++*its;
                    if (r[2] != 0.0) break;
                }
                if (!queue) break;
                pending = j;
            }
            k_backsolve<<<1, 1, 0, s>>>(W.H, m + 1, jend, W.g, W.y);
            k_multiaxpy<<<nblk, 256, 0, s>>>(ipc ? W.Zs : W.V, W.ldv, jend, W.y, 1.0, x, N, nullptr);   // x += V y (Z y)
            // true residual r = rhs - Z x (product in the same tier)
            if ((e = matvec(prec, x, W.z)) != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
            ++*mv;
            k_residual<<<nblk, 256, 0, s>>>(rhs, W.z, W.r, N, W.npart);
            k_finish_norm<<<1, 64, 0, s>>>(W.npart, nblk, W.scal, 3);
            if ((e = fetch(4)) != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
            beta = host[3];
            ++*restarts;
        }
    }
};

}  // namespace
}  // namespace h2

using namespace h2;

extern "C" h2_status h2_gmres_workspace(h2_handle h, const h2_gmres_opts* o, size_t* bytes) {
    if (!handle_live(h)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (!o || !bytes) return handle_fail(H2_ERR_INVALID_ARG, "null argument");
    if (o->restart < 1 || o->restart > 127) return handle_fail(H2_ERR_INVALID_ARG, "restart must be in [1, 127]");
    const DevH2* d = handle_dev(h);
    if (o->precond >= H2_PRECOND_MLP && !h->mlp_params) return handle_fail(H2_ERR_INVALID_ARG, "no MLP attached");
    *bytes = work_layout(int64_t(d->n_vox) * kNcomp, o->restart, nullptr, nullptr, o->precond, d->leaves.n,
                         h->mlp_dims.n_in, h->mlp_dims.n_hidden, h->mlp_dims.n_out);
    return H2_OK;
}

extern "C" h2_status h2_gmres_solve(h2_handle h, const void* b, void* x, const h2_gmres_opts* o, h2_gmres_report* rep,
                                    void* work, size_t work_bytes, void* stream) {
    if (!handle_live(h)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (!b || !x || !o || !rep || !work) return handle_fail(H2_ERR_INVALID_ARG, "null argument");
    if (o->restart < 1 || o->restart > 127) return handle_fail(H2_ERR_INVALID_ARG, "restart must be in [1, 127]");
    if (!(o->tol > 0.0) || o->max_matvec < 1) return handle_fail(H2_ERR_INVALID_ARG, "tol must be > 0 and max_matvec >= 1");
    if (o->precision < H2_FP64 || o->precision > H2_BF16X3) return handle_fail(H2_ERR_INVALID_ARG, "unknown precision");
    if ((reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(x)) % 16)
        return handle_fail(H2_ERR_INVALID_ARG, "misaligned vector");
    const DevH2* d = handle_dev(h);
    if (!d->has_tier[o->precision]) return handle_fail(H2_ERR_INVALID_ARG, "precision tier was not built");
    if (o->precision == H2_BF16X3 && (!h->self_group || !h->batch))
        return handle_fail(H2_ERR_INVALID_ARG, "BF16X3 tier was not built");
    if (o->precond < H2_PRECOND_NONE || o->precond > H2_PRECOND_MLP_RESTART)
        return handle_fail(H2_ERR_INVALID_ARG, "unknown preconditioner");
    if (o->precond == H2_PRECOND_BLOCKDIAG && !h->bd_ready)
        return handle_fail(H2_ERR_INVALID_ARG, "block-diagonal preconditioner not formed (h2_precond_blockdiag)");
    if (o->precond >= H2_PRECOND_MLP && !h->mlp_params) return handle_fail(H2_ERR_INVALID_ARG, "no MLP attached");
    const int64_t N = int64_t(d->n_vox) * kNcomp;
    const int m = o->restart;
    const int pc = o->precond;
    const size_t need = work_layout(N, m, nullptr, nullptr, pc, d->leaves.n, h->mlp_dims.n_in, h->mlp_dims.n_hidden,
                                    h->mlp_dims.n_out);
    if (work_bytes < need) return handle_fail(H2_ERR_OOM, "GMRES workspace too small");
    char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(work) + 255) & ~uintptr_t(255));
    Solver S{};
    S.h = h;
    S.d = d;
    S.lv = handle_levels(h);
    S.s = reinterpret_cast<hipStream_t>(stream);
    S.N = N;
    S.nblk = int(std::min<int64_t>(kDotBlocks, (N + 255) / 256));
    work_layout(N, m, &S.W, base, pc, d->leaves.n, h->mlp_dims.n_in, h->mlp_dims.n_hidden, h->mlp_dims.n_out);
    S.precond = pc;
    if (o->precision == H2_BF16X3) {   // block-GEMM tile for one column (tuned once)
        if (hipMemsetAsync(S.W.lo_in, 0, size_t(N) * 8, S.s) != hipSuccess)
            return handle_fail(H2_ERR_DEVICE, "workspace clear failed");
        h2_status ts = group_autotile(h->self_group, S.W.lo_in, S.W.lo_out, 1, N, S.s);
        if (ts != H2_OK) return ts;
    }
    if (hipHostMalloc((void**)&S.host, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess)
        return handle_fail(H2_ERR_DEVICE, "pinned host allocation failed");
    for (auto& ev : S.ev)
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            for (auto& e2 : S.ev)
                if (e2) (void)hipEventDestroy(e2);
            (void)hipHostFree(S.host);
            return handle_fail(H2_ERR_DEVICE, "event creation failed");
        }
    k_zero_flags<<<1, 64, 0, S.s>>>(S.W.flags);
    *rep = h2_gmres_report{};
    h2_status st;
    const double2* bb = (const double2*)b;
    double2* xx = (double2*)x;
    if (o->precision == H2_FP64) {
        int its, mv, rs;
        double rr;
        st = S.gmres(0, bb, xx, m, o->max_matvec, o->tol, &its, &mv, &rs, &rr, o->use_x0 != 0);
        rep->iterations = its;
        rep->matvecs = mv;
        rep->restarts = rs;
        rep->rel_residual = rr;
        rep->converged = (st == H2_OK);
    } else {
        // iterative refinement: r = b - Z x (FP64), inner GMRES with the low-precision product, x += d
        st = H2_OK;
        hipError_t e = hipSuccess;
        if (!o->use_x0) k_fill<<<S.nblk, 256, 0, S.s>>>(xx, N);
        (void)S.norm_into(bb, 2);
        if ((e = S.fetch(3)) != hipSuccess) st = handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
        const double bnorm = S.host[2];
        if (st == H2_OK && !std::isfinite(bnorm)) st = handle_fail(H2_ERR_NUMERIC, "right-hand side holds NaN or Inf");
        double rel = 0.0;
        if (st == H2_OK && bnorm == 0.0 && o->use_x0) k_fill<<<S.nblk, 256, 0, S.s>>>(xx, N);   // x = 0 solves Z x = 0
        // rhs of the inner solve lives in W.xs (the residual), the correction in W.d
        if (st == H2_OK && bnorm > 0) {
            rel = 1.0;
            if (o->use_x0) {   // residual of the given iterate
                if ((e = launch_matvec(*d, *S.lv, 1, 0, xx, S.W.z, 1, N, S.s)) != hipSuccess)
                    st = handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
                rep->matvecs += 1;
                k_residual<<<S.nblk, 256, 0, S.s>>>(bb, S.W.z, S.W.xs, N, S.W.npart);
                k_finish_norm<<<1, 64, 0, S.s>>>(S.W.npart, S.nblk, S.W.scal, 3);
                if (st == H2_OK && (e = S.fetch(4)) != hipSuccess) st = handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
                rel = S.host[3] / bnorm;
            } else {
                e = hipMemcpyAsync(S.W.xs, bb, N * 16, hipMemcpyDeviceToDevice, S.s);
            }
            int outer = 0;
            while (st == H2_OK) {
                if (rel <= o->tol) break;
                if (outer >= o->max_outer || rep->matvecs >= o->max_matvec) { st = H2_NOT_CONVERGED; break; }
                int its, mv, rs;
                double rr;
                h2_status si = S.gmres(o->precision, S.W.xs, S.W.d, m, o->max_matvec - rep->matvecs, o->inner_tol,
                                       &its, &mv, &rs, &rr);
                if (si < 0) { st = si; break; }
                rep->iterations += its;
                rep->matvecs += mv;
                rep->restarts += rs;
                k_add<<<S.nblk, 256, 0, S.s>>>(xx, S.W.d, N);
                if ((e = launch_matvec(*d, *S.lv, 1, 0, xx, S.W.z, 1, N, S.s)) != hipSuccess) {
                    st = handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
                    break;
                }
                rep->matvecs += 1;
                k_residual<<<S.nblk, 256, 0, S.s>>>(bb, S.W.z, S.W.xs, N, S.W.npart);
                k_finish_norm<<<1, 64, 0, S.s>>>(S.W.npart, S.nblk, S.W.scal, 3);
                if ((e = S.fetch(4)) != hipSuccess) { st = handle_fail(H2_ERR_DEVICE, hipGetErrorString(e)); break; }
                rel = S.host[3] / bnorm;
                if (!std::isfinite(rel)) { st = handle_fail(H2_ERR_NUMERIC, "residual is NaN or Inf"); break; }
                ++outer;
            }
            rep->outer = outer;
        }
        rep->rel_residual = rel;
        rep->converged = (st == H2_OK);
    }
    rep->corrections = S.corrections;
    {   // steps that took the second Gram-Schmidt pass, counted on the device
        int fl[4] = {0, 0, 0, 0};
        if (hipMemcpyAsync(fl, S.W.flags, sizeof(fl), hipMemcpyDeviceToHost, S.s) == hipSuccess &&
            hipStreamSynchronize(S.s) == hipSuccess)
            S.reorth = fl[2];
    }
    rep->reorth = S.reorth;
    if (hipStreamSynchronize(S.s) != hipSuccess && st >= 0) st = handle_fail(H2_ERR_DEVICE, "solve synchronisation failed");
    for (auto& ev : S.ev) (void)hipEventDestroy(ev);
    (void)hipHostFree(S.host);
    return st;
}
