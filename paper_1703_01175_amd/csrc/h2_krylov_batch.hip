// Batched restarted GMRES: n_rhs independent systems Z x_c = b_c advanced in
// lockstep, so that every product is one multi-column H^2 product (the paper's
// many right-hand sides, Sec. IV.D, Sec. V).
//
// Each column keeps its own Krylov basis, Hessenberg matrix, rotations and
// residual estimate; the Arnoldi arithmetic (classical Gram-Schmidt, with a
// second pass for a column whose first pass left less than 1/sqrt(2) of its
// ||w||, and Givens rotations) is FP64 for every product tier.  With the FP32 or
// BF16x3 product the solve is iterative refinement: the outer residual
// b_c - Z x_c is formed with the FP64 product, the inner solve for the
// correction uses the low-precision product, x_c += d_c.  A column whose
// estimate reaches its target (or whose Arnoldi breaks down) keeps moving
// with the others but its basis stops growing: the cycle's update uses only its
// first jend_c vectors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "h2_api_internal.h"
#include "h2_givens.h"

namespace h2 {
namespace {

constexpr int kTile = 16;         // basis vectors per dot-product pass
constexpr int kHs = 128;          // per-column stride of hcol, cs, sn, y
constexpr int kGs = 136;          // per-column stride of g
constexpr int kSs = 8;            // per-column stride of the scalars: 0 ||w||, 1 |g_{j+1}|, 2 ||b||, 3 ||r||,
                                  // 5 ||w|| before orthogonalisation, 6-7 step of the restart correction
constexpr double kDgks = 0.70710678118654752;   // repeat Gram-Schmidt when the norm drops below this fraction

__device__ __forceinline__ double2 cmul_conj(double2 a, double2 b) {   // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// partial[c][blk][i] = this block's share of conj(V_c,i) . w_c, i in [i0, i0 + 16) and i < n_c
// (n_c = nv ? nv[c] : nvec)
__global__ __launch_bounds__(256) void kb_multidot(const double2* __restrict__ V, int64_t ldv, int64_t vs, int nvec,
                                                   const int* __restrict__ nv, const double2* __restrict__ w, int64_t ws,
                                                   int64_t N, double2* __restrict__ partial) {
    __shared__ double2 red[4][kTile];
    const int c = blockIdx.z;
    const double2* Vc = V + c * vs;
    const double2* wc = w + c * ws;
    const int i0 = blockIdx.y * kTile;
    const int cnt = min(kTile, (nv ? nv[c] : nvec) - i0);
    if (cnt <= 0) return;
    double2 acc[kTile];
#pragma unroll
    for (int q = 0; q < kTile; ++q) acc[q] = make_double2(0, 0);
    for (int64_t n = blockIdx.x * 256 + threadIdx.x; n < N; n += int64_t(gridDim.x) * 256) {
        const double2 wv = wc[n];
#pragma unroll
        for (int q = 0; q < kTile; ++q)
            if (q < cnt) {
                const double2 p = cmul_conj(Vc[(int64_t)(i0 + q) * ldv + n], wv);
                acc[q].x += p.x;
                acc[q].y += p.y;
            }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kTile; ++q) {
        const double rx = wsum(acc[q].x), ry = wsum(acc[q].y);
        if (lane == 0) red[wave][q] = make_double2(rx, ry);
    }
    __syncthreads();
    if (threadIdx.x < cnt) {
        const int q = threadIdx.x;
        double2 s = red[0][q];
        for (int k = 1; k < 4; ++k) { s.x += red[k][q].x; s.y += red[k][q].y; }
        partial[((int64_t)c * gridDim.x + blockIdx.x) * 128 + i0 + q] = s;
    }
}

// out[c][i] (+)= sum_blk partial[c][blk][i] for i < n_c, 0 for n_c <= i < nvec (one group of 128 per column)
__global__ void kb_reduce(const double2* __restrict__ partial, int nblk, int nvec, const int* __restrict__ nv,
                          double2* __restrict__ out, int accumulate) {
    const int c = blockIdx.x, i = threadIdx.x;
    if (i >= nvec) return;
    const double2* p = partial + (int64_t)c * nblk * 128;
    double2 s = make_double2(0, 0);
    if (i < (nv ? nv[c] : nvec))
        for (int b = 0; b < nblk; ++b) { s.x += p[(int64_t)b * 128 + i].x; s.y += p[(int64_t)b * 128 + i].y; }
    double2* o = out + (int64_t)c * kHs + i;
    if (accumulate) { s.x += o->x; s.y += o->y; }
    *o = s;
}

// w_c += sign * sum_{i < n_c} V_c,i coef_c,i with n_c = nv ? nv[c] : nvec; optional partial norms
__global__ __launch_bounds__(256) void kb_multiaxpy(const double2* __restrict__ V, int64_t ldv, int64_t vs, int nvec,
                                                    const int* __restrict__ nv, const double2* __restrict__ coef,
                                                    double sign, double2* __restrict__ w, int64_t ws, int64_t N,
                                                    double* __restrict__ npart) {
    __shared__ double2 cs[128];
    __shared__ double red[4];
    const int c = blockIdx.z;
    const int n_c = nv ? nv[c] : nvec;
    const double2* Vc = V + c * vs;
    double2* wc = w + c * ws;
    for (int i = threadIdx.x; i < n_c; i += 256) cs[i] = coef[(int64_t)c * kHs + i];
    __syncthreads();
    double nn = 0;
    for (int64_t n = blockIdx.x * 256 + threadIdx.x; n < N; n += int64_t(gridDim.x) * 256) {
        double2 a = make_double2(0, 0);
        for (int i = 0; i < n_c; ++i) {
            const double2 v = Vc[(int64_t)i * ldv + n];
            const double2 ci = cs[i];
            a.x = fma(v.x, ci.x, a.x);
            a.x = fma(-v.y, ci.y, a.x);
            a.y = fma(v.x, ci.y, a.y);
            a.y = fma(v.y, ci.x, a.y);
        }
        double2 r = wc[n];
        r.x += sign * a.x;
        r.y += sign * a.y;
        wc[n] = r;
        nn += r.x * r.x + r.y * r.y;
    }
    if (npart) {
        nn = wsum(nn);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
        __syncthreads();
        if (threadIdx.x == 0) npart[(int64_t)c * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

// r_c = b_c - z_c, partial norms
__global__ __launch_bounds__(256) void kb_residual(const double2* __restrict__ b, int64_t bs, const double2* __restrict__ z,
                                                   int64_t zs, double2* __restrict__ r, int64_t rs, int64_t N,
                                                   double* __restrict__ npart) {
    __shared__ double red[4];
    const int c = blockIdx.z;
    double nn = 0;
    for (int64_t n = blockIdx.x * 256 + threadIdx.x; n < N; n += int64_t(gridDim.x) * 256) {
        const double2 bv = b[c * bs + n], zv = z[c * zs + n];
        const double2 v = make_double2(bv.x - zv.x, bv.y - zv.y);
        r[c * rs + n] = v;
        nn += v.x * v.x + v.y * v.y;
    }
    nn = wsum(nn);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
    __syncthreads();
    if (threadIdx.x == 0) npart[(int64_t)c * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void kb_norm2(const double2* __restrict__ a, int64_t as, int64_t N,
                                                double* __restrict__ npart) {
    __shared__ double red[4];
    const int c = blockIdx.z;
    double nn = 0;
    for (int64_t n = blockIdx.x * 256 + threadIdx.x; n < N; n += int64_t(gridDim.x) * 256) {
        const double2 v = a[c * as + n];
        nn += v.x * v.x + v.y * v.y;
    }
    nn = wsum(nn);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
    __syncthreads();
    if (threadIdx.x == 0) npart[(int64_t)c * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// scal[c][slot] = sqrt(sum of the column's partials), fixed order
__global__ void kb_finish_norm(const double* __restrict__ npart, int nblk, double* __restrict__ scal, int slot) {
    const int c = blockIdx.x;
    double s = 0;
    for (int b = threadIdx.x; b < nblk; b += 64) s += npart[(int64_t)c * nblk + b];
    s = wsum(s);
    if (threadIdx.x == 0) scal[c * kSs + slot] = sqrt(s);
}

// dst_c = src_c / scal[c][slot]  (zeros where that norm is zero: an exhausted column)
__global__ void kb_scale(const double2* __restrict__ src, int64_t ss, double2* __restrict__ dst, int64_t ds, int64_t N,
                         const double* __restrict__ scal, int slot) {
    const int c = blockIdx.z;
    const double nv = scal[c * kSs + slot];
    const double inv = nv > 0.0 ? 1.0 / nv : 0.0;
    for (int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; n < N; n += int64_t(gridDim.x) * blockDim.x) {
        const double2 v = src[c * ss + n];
        dst[c * ds + n] = make_double2(v.x * inv, v.y * inv);
    }
}

__global__ void kb_fill(double2* __restrict__ a, int64_t as, int64_t N) {
    const int c = blockIdx.z;
    for (int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; n < N; n += int64_t(gridDim.x) * blockDim.x)
        a[c * as + n] = make_double2(0, 0);
}

// x_c += d_c where live[c]
__global__ void kb_add(double2* __restrict__ x, int64_t xs, const double2* __restrict__ d, int64_t ds, int64_t N,
                       const int* __restrict__ live) {
    const int c = blockIdx.z;
    if (!live[c]) return;
    for (int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; n < N; n += int64_t(gridDim.x) * blockDim.x) {
        x[c * xs + n].x += d[c * ds + n].x;
        x[c * xs + n].y += d[c * ds + n].y;
    }
}

// zero the columns that are not live (their inner right-hand side)
__global__ void kb_mask(double2* __restrict__ a, int64_t as, int64_t N, const int* __restrict__ live) {
    const int c = blockIdx.z;
    if (live[c]) return;
    for (int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; n < N; n += int64_t(gridDim.x) * blockDim.x)
        a[c * as + n] = make_double2(0, 0);
}

// a[c][i] += b[c][i], i < n
__global__ void kb_reduce_add(double2* __restrict__ a, const double2* __restrict__ b, int n) {
    const int c = blockIdx.x, i = threadIdx.x;
    if (i >= n) return;
    a[(int64_t)c * kHs + i].x += b[(int64_t)c * kHs + i].x;
    a[(int64_t)c * kHs + i].y += b[(int64_t)c * kHs + i].y;
}



__global__ void kb_givens(double2* __restrict__ H, int64_t hs, int ldh, int j, const double2* __restrict__ hcol,
                          double* __restrict__ cs, double2* __restrict__ sn, double2* __restrict__ g,
                          double* __restrict__ scal) {
    if (threadIdx.x != 0) return;
    const int c = blockIdx.x;
    double2* col = H + c * hs + (int64_t)j * ldh;
    for (int i = 0; i <= j; ++i) col[i] = hcol[(int64_t)c * kHs + i];
    col[j + 1] = make_double2(scal[c * kSs + 0], 0.0);
    scal[c * kSs + 1] = givens_column(col, j, cs + (int64_t)c * kHs, sn + (int64_t)c * kHs, g + (int64_t)c * kGs);
}

__global__ void kb_backsolve(const double2* __restrict__ H, int64_t hs, int ldh, const int* __restrict__ jend,
                             const double2* __restrict__ g, double2* __restrict__ y) {
    if (threadIdx.x != 0) return;
    const int c = blockIdx.x;
    back_substitute(H + c * hs, ldh, jend[c], g + (int64_t)c * kGs, y + (int64_t)c * kHs);
}

__global__ void kb_init_g(double2* __restrict__ g, int m, const double* __restrict__ scal, int slot) {
    const int c = blockIdx.x;
    for (int i = threadIdx.x; i <= m; i += blockDim.x)
        g[(int64_t)c * kGs + i] = make_double2(i == 0 ? scal[c * kSs + slot] : 0.0, 0.0);
}

// Restart correction, per column: scal[c][6..7] = alpha_c = w^H r / ||w||^2 from the dot
// (dots[c]) and the partial norms of w; 0 for a column that is not open, when ||w|| = 0,
// or when alpha is not a number.
__global__ void kb_mr_alpha(const double* __restrict__ npart, int nblk, const double2* __restrict__ dots,
                            double* __restrict__ scal, const int* __restrict__ open) {
    const int c = blockIdx.x;
    double s = 0;
    for (int b = threadIdx.x; b < nblk; b += 64) s += npart[(int64_t)c * nblk + b];
    s = wsum(s);
    if (threadIdx.x == 0) {
        double ar = 0.0, ai = 0.0;
        if (open[c] && s > 0.0) {
            ar = dots[(int64_t)c * kHs].x / s;
            ai = dots[(int64_t)c * kHs].y / s;
            if (!isfinite(ar) || !isfinite(ai)) ar = ai = 0.0;
        }
        scal[c * kSs + 6] = ar;
        scal[c * kSs + 7] = ai;
    }
}

// d_c += alpha_c c_c, r_c -= alpha_c w_c; partial squared norms of the new r_c
__global__ __launch_bounds__(256) void kb_mr_step(double2* __restrict__ d, const double2* __restrict__ cv,
                                                  double2* __restrict__ r, const double2* __restrict__ w, int64_t ld,
                                                  int64_t N, const double* __restrict__ scal,
                                                  double* __restrict__ npart) {
    __shared__ double red[4];
    const int c = blockIdx.z;
    const double ar = scal[c * kSs + 6], ai = scal[c * kSs + 7];
    double nn = 0;
    for (int64_t n = blockIdx.x * 256 + threadIdx.x; n < N; n += int64_t(gridDim.x) * 256) {
        const int64_t o = c * ld + n;
        const double2 a = cv[o], wv = w[o];
        double2 dv = d[o], rv = r[o];
        dv.x += ar * a.x - ai * a.y;
        dv.y += ar * a.y + ai * a.x;
        rv.x -= ar * wv.x - ai * wv.y;
        rv.y -= ar * wv.y + ai * wv.x;
        d[o] = dv;
        r[o] = rv;
        nn += rv.x * rv.x + rv.y * rv.y;
    }
    nn = wsum(nn);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
    __syncthreads();
    if (threadIdx.x == 0) npart[(int64_t)c * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

struct BWork {
    double2 *V, *Zs;                 // bases [j][c][ld]
    double2 *W, *Rin, *R, *D, *Zx;   // columns [c][ld]
    float2 *lo_in, *lo_out;
    double2 *hcol, *H, *sn, *g, *y, *dpart;
    double *cs, *scal, *npart;
    int *jend, *live, *acc;
    float *mX, *mH1, *mH2, *mY;
    double* mnorm;
};

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

size_t bwork_layout(int64_t ld, int ncol, int m, int nblk, BWork* W, char* base, int precond, int64_t nleaf,
                    int n_in, int n_hidden, int n_out) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += al256(bytes);
        return p;
    };
    const size_t col = size_t(ld) * ncol;
    BWork w{};
    w.V = (double2*)take(col * (m + 1) * 16);
    w.Zs = precond ? (double2*)take(col * m * 16) : nullptr;
    if (precond >= 2) {
        w.mX = (float*)take(size_t(nleaf) * n_in * 4);
        w.mH1 = (float*)take(size_t(nleaf) * n_hidden * 4);
        w.mH2 = (float*)take(size_t(nleaf) * n_hidden * 4);
        w.mY = (float*)take(size_t(nleaf) * n_out * 4);
        w.mnorm = (double*)take(64);
    }
    w.W = (double2*)take(col * 16);
    w.Rin = (double2*)take(col * 16);
    w.R = (double2*)take(col * 16);
    w.D = (double2*)take(col * 16);
    w.Zx = (double2*)take(col * 16);
    w.lo_in = (float2*)take(col * 8);
    w.lo_out = (float2*)take(col * 8);
    w.hcol = (double2*)take(size_t(ncol) * kHs * 16);
    w.H = (double2*)take(size_t(ncol) * (m + 1) * m * 16);
    w.cs = (double*)take(size_t(ncol) * kHs * 8);
    w.sn = (double2*)take(size_t(ncol) * kHs * 16);
    w.g = (double2*)take(size_t(ncol) * kGs * 16);
    w.y = (double2*)take(size_t(ncol) * kHs * 16);
    w.scal = (double*)take(size_t(ncol) * kSs * 8);
    w.npart = (double*)take(size_t(ncol) * nblk * 8);
    w.dpart = (double2*)take(size_t(ncol) * nblk * 128 * 16);
    w.jend = (int*)take(size_t(ncol) * 4);
    w.live = (int*)take(size_t(ncol) * 4);
    w.acc = (int*)take(size_t(ncol) * 4);
    if (W) *W = w;
    return off + 256;
}

int blocks_per_column(int64_t N, int ncol) {
    const int64_t want = std::max<int64_t>(16, 2048 / std::max(ncol, 1));
    return int(std::min<int64_t>(want, (N + 255) / 256));
}

struct BSolver {
    h2_handle h;
    const DevH2* d;
    const LevelLaunch* lv;
    hipStream_t s;
    int64_t N, ld;
    int ncol, m, nblk, precond;
    BWork W;
    double* host = nullptr;        // pinned: ncol * kSs doubles
    std::vector<int> hjend, hlive;

    dim3 cgrid() const { return dim3(nblk, 1, ncol); }

    // y_c = Z x_c for all columns (product tier prec), columns of stride ld
    h2_status prod(int prec, const double2* x, double2* y) {
        hipError_t e;
        if (prec == H2_FP64) {
            e = launch_matvec_multi(*d, *lv, 1, 0, x, y, ncol, ld, s);
            return e == hipSuccess ? H2_OK : handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
        }
        const int64_t flat = ld * ncol;
        if ((e = launch_vec_to_fp32(x, W.lo_in, flat, s)) != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
        if (prec == H2_FP32) {
            e = launch_matvec_multi(*d, *lv, 1, 1, W.lo_in, W.lo_out, ncol, ld, s);
            if (e != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
        } else {
            const void* xin[1] = {W.lo_in};
            void* yout[1] = {W.lo_out};
            const int64_t nr[1] = {ncol}, lds[1] = {ld};
            h2_status st = group_run(h->self_group, 1, xin, yout, nr, lds, s);
            if (st != H2_OK) return st;
        }
        if ((e = launch_vec_to_fp64(W.lo_out, y, flat, s)) != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
        return H2_OK;
    }

    // Arnoldi's right preconditioner: 0 none, 1 block diagonal, 2 MLP; the restart
    // correction (3) runs its cycles with the MLP's base map.
    int inner_pc() const { return precond == 3 ? (h->mlp_base == H2_PRECOND_BLOCKDIAG ? 1 : 0) : precond; }

    h2_status precondition(const double2* v, double2* z) {   // z_c = P(v_c), column by column
        for (int c = 0; c < ncol; ++c) {
            hipError_t e;
            if (inner_pc() == H2_PRECOND_BLOCKDIAG)
                e = launch_bd_apply(d->leaves, d->perm, (const double2*)h->bd_buf, v + c * ld, z + c * ld, s);
            else
                e = mlp_apply_handle(h, v + c * ld, z + c * ld, W.mX, W.mH1, W.mH2, W.mY, W.mnorm, s);
            if (e != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
        }
        return H2_OK;
    }

    void norms(const double2* a, int slot) {
        kb_norm2<<<cgrid(), 256, 0, s>>>(a, ld, N, W.npart);
        kb_finish_norm<<<ncol, 64, 0, s>>>(W.npart, nblk, W.scal, slot);
    }

    h2_status fetch() {
        hipError_t e = hipMemcpyAsync(host, W.scal, size_t(ncol) * kSs * 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e == hipSuccess ? H2_OK : handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
    }

    h2_status upload_ints(int* dev, const std::vector<int>& v) {
        hipError_t e = hipMemcpyAsync(dev, v.data(), size_t(ncol) * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);   // v is pageable host memory
        return e == hipSuccess ? H2_OK : handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
    }

    // Learned correction at a cycle start, per open column: c = P(r_c), w = Z c and the
    // minimal-residual step d_c += alpha_c c, r_c -= alpha_c w with alpha_c = w^H r_c / ||w||^2
    // (none when w = 0); res follows r.
    h2_status restart_correction(int prec, double2* dsol, std::vector<double>& res, const std::vector<char>& open,
                                 std::vector<int>& mv, int* spent) {
        hipError_t e;
        for (int c = 0; c < ncol; ++c) {
            if (open[c])
                e = mlp_apply_handle(h, W.Rin + c * ld, W.W + c * ld, W.mX, W.mH1, W.mH2, W.mY, W.mnorm, s);
            else
                e = hipMemsetAsync(W.W + c * ld, 0, size_t(N) * 16, s);
            if (e != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
        }
        h2_status st = prod(prec, W.W, W.Zx);
        if (st != H2_OK) return st;
        ++*spent;
        std::vector<int> op(ncol, 0);
        for (int c = 0; c < ncol; ++c) op[c] = open[c] ? 1 : 0;
        if ((st = upload_ints(W.acc, op)) != H2_OK) return st;
        kb_multidot<<<cgrid(), 256, 0, s>>>(W.Zx, ld, ld, 1, nullptr, W.Rin, ld, N, W.dpart);   // w^H r
        kb_reduce<<<ncol, 128, 0, s>>>(W.dpart, nblk, 1, nullptr, W.y, 0);
        kb_norm2<<<cgrid(), 256, 0, s>>>(W.Zx, ld, N, W.npart);                                 // ||w||^2
        kb_mr_alpha<<<ncol, 64, 0, s>>>(W.npart, nblk, W.y, W.scal, W.acc);
        kb_mr_step<<<cgrid(), 256, 0, s>>>(dsol, W.W, W.Rin, W.Zx, ld, N, W.scal, W.npart);
        kb_finish_norm<<<ncol, 64, 0, s>>>(W.npart, nblk, W.scal, 3);
        if ((st = fetch()) != H2_OK) return st;
        for (int c = 0; c < ncol; ++c) {
            if (!open[c]) continue;
            ++mv[c];
            if (host[c * kSs + 6] != 0.0 || host[c * kSs + 7] != 0.0) {
                ++corrections[c];
                res[c] = host[c * kSs + 3];
            }
        }
        return H2_OK;
    }
    std::vector<int> corrections;
    std::vector<int> reorth;           // per column: Arnoldi steps that repeated Gram-Schmidt

    void multidot(int nvec, const double2* w, double2* out, int accumulate, const int* nv = nullptr) {   // basis [j][c][ld]
        dim3 grid(nblk, (nvec + kTile - 1) / kTile, ncol);
        kb_multidot<<<grid, 256, 0, s>>>(W.V, ld * ncol, ld, nvec, nv, w, ld, N, W.dpart);
        kb_reduce<<<ncol, 128, 0, s>>>(W.dpart, nblk, nvec, nv, out, accumulate);
    }

    // Restarted GMRES on Z d_c = rhs_c from d = 0 for the live columns, until
    // ||rhs_c - Z d_c|| <= target_c (absolute) or the budget is spent; the
    // product is tier prec.  its/mv/restarts count per column (lockstep).
    // On return Rin holds rhs - Z d and scal[c][3] its norm.
    h2_status inner(int prec, const double2* rhs, double2* dsol, const std::vector<double>& target, int max_mv,
                    std::vector<int>& its, std::vector<int>& mv, std::vector<int>& restarts, std::vector<double>& res,
                    int* used_mv) {
        h2_status st;
        kb_fill<<<cgrid(), 256, 0, s>>>(dsol, ld, N);
        hipError_t e = hipMemcpyAsync(W.Rin, rhs, size_t(ld) * ncol * 16, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
        norms(W.Rin, 3);
        if ((st = fetch()) != H2_OK) return st;
        std::vector<char> open(ncol);
        for (int c = 0; c < ncol; ++c) res[c] = host[c * kSs + 3];
        int spent = 0;
        const int ipc = inner_pc();
        while (true) {
            bool any = false;
            for (int c = 0; c < ncol; ++c) {
                open[c] = hlive[c] && res[c] > target[c] && std::isfinite(res[c]);
                any = any || open[c];
            }
            if (!any || spent >= max_mv) break;
            if (precond == 3) {
                if ((st = restart_correction(prec, dsol, res, open, mv, &spent)) != H2_OK) return st;
                any = false;
                for (int c = 0; c < ncol; ++c) {
                    open[c] = open[c] && res[c] > target[c];
                    any = any || open[c];
                }
                if (!any || spent >= max_mv) break;
            }
            // v_0 = r / ||r|| (columns that are not open start from zero and stay there)
            for (int c = 0; c < ncol; ++c) host[c * kSs + 3] = open[c] ? res[c] : 0.0;
            if ((e = hipMemcpyAsync(W.scal, host, size_t(ncol) * kSs * 8, hipMemcpyHostToDevice, s)) != hipSuccess)
                return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
            kb_scale<<<cgrid(), 256, 0, s>>>(W.Rin, ld, W.V, ld, N, W.scal, 3);
            kb_init_g<<<ncol, 256, 0, s>>>(W.g, m, W.scal, 3);
            std::vector<char> grow(open);
            std::fill(hjend.begin(), hjend.end(), 0);
            const int64_t blk = ld * ncol;               // one basis vector of every column
            for (int j = 0; j < m; ++j) {
                const double2* vj = W.V + (int64_t)j * blk;
                const double2* src = vj;
                if (ipc) {
                    double2* zj = W.Zs + (int64_t)j * blk;
                    if ((st = precondition(vj, zj)) != H2_OK) return st;
                    src = zj;
                }
                if ((st = prod(prec, src, W.W)) != H2_OK) return st;
                ++spent;
                for (int c = 0; c < ncol; ++c)
                    if (grow[c]) { ++its[c]; ++mv[c]; }
                // classical Gram-Schmidt; a column repeats it when its norm fell below 1/sqrt(2)
                // of ||w|| (the Daniel-Gragg-Kaufman-Stewart test), the others keep one pass
                norms(W.W, 5);
                multidot(j + 1, W.W, W.hcol, 0);
                kb_multiaxpy<<<cgrid(), 256, 0, s>>>(W.V, blk, ld, j + 1, nullptr, W.hcol, -1.0, W.W, ld, N, W.npart);
                kb_finish_norm<<<ncol, 64, 0, s>>>(W.npart, nblk, W.scal, 0);
                if ((st = fetch()) != H2_OK) return st;
                std::vector<int> again(ncol, 0);
                bool any_again = false;
                for (int c = 0; c < ncol; ++c)
                    if (grow[c] && !(host[c * kSs + 0] >= kDgks * host[c * kSs + 5])) {
                        again[c] = j + 1;
                        any_again = true;
                        ++reorth[c];
                    }
                if (any_again) {
                    if ((st = upload_ints(W.acc, again)) != H2_OK) return st;
                    multidot(j + 1, W.W, W.y, 0, W.acc);     // second pass (y as scratch, zeros elsewhere)
                    kb_multiaxpy<<<cgrid(), 256, 0, s>>>(W.V, blk, ld, j + 1, W.acc, W.y, -1.0, W.W, ld, N, W.npart);
                    kb_reduce_add<<<ncol, 128, 0, s>>>(W.hcol, W.y, j + 1);
                    kb_finish_norm<<<ncol, 64, 0, s>>>(W.npart, nblk, W.scal, 0);
                }
                kb_givens<<<ncol, 64, 0, s>>>(W.H, int64_t(m + 1) * m, m + 1, j, W.hcol, W.cs, W.sn, W.g, W.scal);
                if ((st = fetch()) != H2_OK) return st;
                bool more = false;
                for (int c = 0; c < ncol; ++c) {
                    if (!grow[c]) continue;
                    hjend[c] = j + 1;
                    const double hn = host[c * kSs + 0], est = host[c * kSs + 1];
                    if (!std::isfinite(est)) return handle_fail(H2_ERR_NUMERIC, "residual estimate is NaN or Inf");
                    if (hn == 0.0 || est <= target[c]) grow[c] = 0;
                    more = more || grow[c];
                }
                if (!more || spent >= max_mv) break;
                kb_scale<<<cgrid(), 256, 0, s>>>(W.W, ld, W.V + (int64_t)(j + 1) * blk, ld, N, W.scal, 0);
            }
            // d_c += basis_c y_c over the column's own jend_c vectors
            if ((st = upload_ints(W.jend, hjend)) != H2_OK) return st;
            kb_backsolve<<<ncol, 64, 0, s>>>(W.H, int64_t(m + 1) * m, m + 1, W.jend, W.g, W.y);
            kb_multiaxpy<<<cgrid(), 256, 0, s>>>(ipc ? W.Zs : W.V, blk, ld, m, W.jend, W.y, 1.0, dsol, ld, N,
                                                nullptr);
            // true inner residual rhs - Z d in the same tier
            if ((st = prod(prec, dsol, W.Zx)) != H2_OK) return st;
            ++spent;
            for (int c = 0; c < ncol; ++c)
                if (open[c]) { ++mv[c]; ++restarts[c]; }
            kb_residual<<<cgrid(), 256, 0, s>>>(rhs, ld, W.Zx, ld, W.Rin, ld, N, W.npart);
            kb_finish_norm<<<ncol, 64, 0, s>>>(W.npart, nblk, W.scal, 3);
            if ((st = fetch()) != H2_OK) return st;
            for (int c = 0; c < ncol; ++c)
                if (open[c]) res[c] = host[c * kSs + 3];
        }
        *used_mv = spent;
        return H2_OK;
    }
};

}  // namespace
}  // namespace h2

using namespace h2;

static h2_status batch_check(h2_handle h, int64_t n_rhs, int64_t ld, const h2_gmres_opts* o) {
    if (!handle_live(h)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (!o) return handle_fail(H2_ERR_INVALID_ARG, "null options");
    const int64_t N = int64_t(h->dev.n_vox) * kNcomp;
    if (n_rhs < 1 || n_rhs > 1024) return handle_fail(H2_ERR_INVALID_ARG, "n_rhs must be in [1, 1024]");
    if (ld < N) return handle_fail(H2_ERR_INVALID_ARG, "ld must be >= N");
    if (o->restart < 1 || o->restart > 127) return handle_fail(H2_ERR_INVALID_ARG, "restart must be in [1, 127]");
    if (!(o->tol > 0.0) || o->max_matvec < 1) return handle_fail(H2_ERR_INVALID_ARG, "tol must be > 0 and max_matvec >= 1");
    if (o->precision < H2_FP64 || o->precision > H2_BF16X3) return handle_fail(H2_ERR_INVALID_ARG, "unknown precision");
    if (!h->dev.has_tier[o->precision]) return handle_fail(H2_ERR_INVALID_ARG, "precision tier was not built");
    if (o->precision == H2_BF16X3) {
        if (!h->self_group || !h->batch) return handle_fail(H2_ERR_INVALID_ARG, "BF16X3 tier was not built");
        if (n_rhs * kNcomp > h->batch->max_cols) return handle_fail(H2_ERR_INVALID_ARG, "n_rhs above the built max_rhs");
    }
    if (o->precision != H2_FP64 && !(o->inner_tol > 0.0 && o->inner_tol < 1.0))
        return handle_fail(H2_ERR_INVALID_ARG, "inner_tol must be in (0, 1)");
    if (o->precond < H2_PRECOND_NONE || o->precond > H2_PRECOND_MLP_RESTART)
        return handle_fail(H2_ERR_INVALID_ARG, "unknown preconditioner");
    if (o->precond == H2_PRECOND_BLOCKDIAG && !h->bd_ready)
        return handle_fail(H2_ERR_INVALID_ARG, "block-diagonal preconditioner not formed (h2_precond_blockdiag)");
    if (o->precond >= H2_PRECOND_MLP && !h->mlp_params) return handle_fail(H2_ERR_INVALID_ARG, "no MLP attached");
    return H2_OK;
}

static size_t batch_bytes(h2_handle h, int64_t n_rhs, int64_t ld, const h2_gmres_opts* o, int* nblk) {
    const int64_t N = int64_t(h->dev.n_vox) * kNcomp;
    *nblk = blocks_per_column(N, int(n_rhs));
    return bwork_layout(ld, int(n_rhs), o->restart, *nblk, nullptr, nullptr, o->precond, h->dev.leaves.n,
                        h->mlp_dims.n_in, h->mlp_dims.n_hidden, h->mlp_dims.n_out);
}

extern "C" h2_status h2_gmres_batch_workspace(h2_handle h, int64_t n_rhs, int64_t ld, const h2_gmres_opts* o,
                                              size_t* bytes) {
    h2_status st = batch_check(h, n_rhs, ld, o);
    if (st != H2_OK) return st;
    if (!bytes) return handle_fail(H2_ERR_INVALID_ARG, "null argument");
    int nblk;
    *bytes = batch_bytes(h, n_rhs, ld, o, &nblk);
    return H2_OK;
}

extern "C" h2_status h2_gmres_solve_batch(h2_handle h, int64_t n_rhs, const void* b, void* x, int64_t ld,
                                          const h2_gmres_opts* o, h2_gmres_report* reps, void* work, size_t work_bytes,
                                          void* stream) {
    h2_status st = batch_check(h, n_rhs, ld, o);
    if (st != H2_OK) return st;
    if (!b || !x || !reps || !work) return handle_fail(H2_ERR_INVALID_ARG, "null argument");
    if ((reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(x)) % 16)
        return handle_fail(H2_ERR_INVALID_ARG, "b and x must be 16-byte aligned");
    int nblk;
    const size_t need = batch_bytes(h, n_rhs, ld, o, &nblk);
    if (work_bytes < need) return handle_fail(H2_ERR_OOM, "batched GMRES workspace too small");
    const int ncol = int(n_rhs);
    BSolver S{};
    S.h = h;
    S.d = &h->dev;
    S.lv = &h->lv;
    S.s = reinterpret_cast<hipStream_t>(stream);
    S.N = int64_t(h->dev.n_vox) * kNcomp;
    S.ld = ld;
    S.ncol = ncol;
    S.m = o->restart;
    S.nblk = nblk;
    S.precond = o->precond;
    char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(work) + 255) & ~uintptr_t(255));
    bwork_layout(ld, ncol, S.m, nblk, &S.W, base, o->precond, h->dev.leaves.n, h->mlp_dims.n_in, h->mlp_dims.n_hidden,
                 h->mlp_dims.n_out);
    if (hipHostMalloc((void**)&S.host, size_t(ncol) * kSs * 8, hipHostMallocDefault) != hipSuccess)
        return handle_fail(H2_ERR_DEVICE, "pinned host allocation failed");
    S.hjend.assign(ncol, 0);
    S.corrections.assign(ncol, 0);
    S.reorth.assign(ncol, 0);
    S.hlive.assign(ncol, 1);
    const double2* B = reinterpret_cast<const double2*>(b);
    double2* X = reinterpret_cast<double2*>(x);
    std::vector<int> its(ncol, 0), mv(ncol, 0), rs(ncol, 0), outer(ncol, 0);
    std::vector<double> bn(ncol), rel(ncol, 0.0), res(ncol), target(ncol);
    const int prec = o->precision;
    int spent = 0;

    auto run = [&]() -> h2_status {
        h2_status st2;
        const dim3 cg = S.cgrid();
        if (prec == H2_BF16X3) {   // block-GEMM tile for this column count (tuned once per count)
            if (hipMemsetAsync(S.W.lo_in, 0, size_t(ld) * ncol * 8, S.s) != hipSuccess)
                return handle_fail(H2_ERR_DEVICE, "workspace clear failed");
            if ((st2 = group_autotile(h->self_group, S.W.lo_in, S.W.lo_out, ncol, ld, S.s)) != H2_OK) return st2;
        }
        S.norms(B, 2);
        if ((st2 = S.fetch()) != H2_OK) return st2;
        for (int c = 0; c < ncol; ++c) {
            bn[c] = S.host[c * kSs + 2];
            if (!std::isfinite(bn[c])) return handle_fail(H2_ERR_NUMERIC, "a right-hand side holds NaN or Inf");
        }
        // R = B - Z X0 (FP64), or R = B from X0 = 0
        if (o->use_x0) {
            if ((st2 = S.prod(H2_FP64, X, S.W.Zx)) != H2_OK) return st2;
            ++spent;
            for (int c = 0; c < ncol; ++c) ++mv[c];
            kb_residual<<<cg, 256, 0, S.s>>>(B, ld, S.W.Zx, ld, S.W.R, ld, S.N, S.W.npart);
            kb_finish_norm<<<ncol, 64, 0, S.s>>>(S.W.npart, nblk, S.W.scal, 3);
            if ((st2 = S.fetch()) != H2_OK) return st2;
            for (int c = 0; c < ncol; ++c) res[c] = S.host[c * kSs + 3];
        } else {
            kb_fill<<<cg, 256, 0, S.s>>>(X, ld, S.N);
            hipError_t e = hipMemcpy2DAsync(S.W.R, ld * 16, B, ld * 16, S.N * 16, ncol, hipMemcpyDeviceToDevice, S.s);
            if (e != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
            res = bn;
        }
        for (int c = 0; c < ncol; ++c) rel[c] = bn[c] > 0 ? res[c] / bn[c] : 0.0;
        for (int round = 0;; ++round) {
            bool any = false;
            for (int c = 0; c < ncol; ++c) {
                S.hlive[c] = bn[c] > 0 && rel[c] > o->tol;
                any = any || S.hlive[c];
            }
            if (!any) break;
            if (round >= (prec == H2_FP64 ? 1 : o->max_outer) || spent >= o->max_matvec) break;
            if ((st2 = S.upload_ints(S.W.live, S.hlive)) != H2_OK) return st2;
            kb_mask<<<cg, 256, 0, S.s>>>(S.W.R, ld, S.N, S.W.live);
            // FP64: one restarted GMRES to the final tolerance; otherwise the inner tolerance
            for (int c = 0; c < ncol; ++c) target[c] = prec == H2_FP64 ? o->tol * bn[c] : o->inner_tol * res[c];
            std::vector<double> ires(ncol, 0.0);
            int used = 0;
            if ((st2 = S.inner(prec, S.W.R, S.W.D, target, o->max_matvec - spent, its, mv, rs, ires, &used)) != H2_OK)
                return st2;
            spent += used;
            kb_add<<<cg, 256, 0, S.s>>>(X, ld, S.W.D, ld, S.N, S.W.live);
            if (prec == H2_FP64) {
                for (int c = 0; c < ncol; ++c)
                    if (S.hlive[c]) { res[c] = ires[c]; rel[c] = res[c] / bn[c]; }
            } else {
                // outer residual in FP64
                if ((st2 = S.prod(H2_FP64, X, S.W.Zx)) != H2_OK) return st2;
                ++spent;
                kb_residual<<<cg, 256, 0, S.s>>>(B, ld, S.W.Zx, ld, S.W.R, ld, S.N, S.W.npart);
                kb_finish_norm<<<ncol, 64, 0, S.s>>>(S.W.npart, nblk, S.W.scal, 3);
                if ((st2 = S.fetch()) != H2_OK) return st2;
                for (int c = 0; c < ncol; ++c)
                    if (S.hlive[c]) {
                        ++mv[c];
                        ++outer[c];
                        res[c] = S.host[c * kSs + 3];
                        rel[c] = res[c] / bn[c];
                        if (!std::isfinite(rel[c])) return handle_fail(H2_ERR_NUMERIC, "residual is NaN or Inf");
                    }
            }
        }
        return H2_OK;
    };
    st = run();
    if (hipStreamSynchronize(S.s) != hipSuccess && st >= 0) st = handle_fail(H2_ERR_DEVICE, "solve synchronisation failed");
    (void)hipHostFree(S.host);
    if (st < 0) return st;
    bool all = true;
    for (int c = 0; c < ncol; ++c) {
        h2_gmres_report& r = reps[c];
        r = h2_gmres_report{};
        r.converged = rel[c] <= o->tol;
        r.iterations = its[c];
        r.matvecs = mv[c];
        r.restarts = rs[c];
        r.outer = outer[c];
        r.rel_residual = rel[c];
        r.corrections = S.corrections[c];
        r.reorth = S.reorth[c];
        all = all && r.converged;
    }
    return all ? H2_OK : H2_NOT_CONVERGED;
}
