// Learned per-leaf preconditioner and block-diagonal fallback.
//
// One MLP (two hidden layers, ReLU) with weights shared by every leaf maps a
// leaf's residual to a leaf correction:
//   x = [Re r_t / s, Im r_t / s, Re chi_t] (voxel-major, zero padded to n_pad voxels),
//   y = W3 relu(W2 relu(W1 x + b1) + b2) + b3,  z_t = (y_re + j y_im) * s,
// with s = ||r|| / sqrt(N).  Training minimises 0.5/n sum ||y - t||^2 by Adam on
// FP32 master weights; forward and backward use the master weights rounded to
// bfloat16.  The fallback solves every leaf's diagonal block exactly:
// z_t = (I + sigma k^2 V G_tt diag(chi_t))^-1 r_t on each component.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "h2_api_internal.h"

namespace h2 {

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
__device__ __forceinline__ float ldv(const float* p) { return *p; }
__device__ __forceinline__ float ldv(const uint16_t* p) { return bf2f(*p); }

// C(i, j) (+)= sum_k A(i, k) B(k, j), A(i, k) = A[i sa0 + k sa1], B(k, j) = B[k sb0 + j sb1];
// epilogue: + bias[j], relu, * (mask(i, j) > 0).  64 x 64 tiles, 16-deep K chunks in LDS.
template <typename TA, typename TB>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const TA* __restrict__ A, int64_t sa0, int64_t sa1,
                                              const TB* __restrict__ B, int64_t sb0, int64_t sb1, float* __restrict__ C,
                                              int64_t ldc, const float* __restrict__ bias, int relu,
                                              const float* __restrict__ mask, int64_t ldm, int accumulate) {
    __shared__ float As[16][65];
    __shared__ float Bs[16][65];
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += 16) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int kk = e >> 6, ii = e & 63;
            const int gi = i0 + ii, gk = k0 + kk, gj = j0 + ii;
            As[kk][ii] = (gi < M && gk < K) ? ldv(A + gi * sa0 + gk * sa1) : 0.f;
            Bs[kk][ii] = (gj < N && gk < K) ? ldv(B + gk * sb0 + gj * sb1) : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = As[kk][ty * 4 + q];
                b[q] = Bs[kk][tx * 4 + q];
            }
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[p][q] = fmaf(a[p], b[q], acc[p][q]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int i = i0 + ty * 4 + p;
        if (i >= M) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = j0 + tx * 4 + q;
            if (j >= N) continue;
            float v = acc[p][q];
            if (accumulate) v += C[i * ldc + j];
            if (bias) v += bias[j];
            if (relu) v = fmaxf(v, 0.f);
            if (mask && !(mask[i * ldm + j] > 0.f)) v = 0.f;
            C[i * ldc + j] = v;
        }
    }
}

template <typename TA, typename TB>
static void gemm(hipStream_t s, int M, int N, int K, const TA* A, int64_t sa0, int64_t sa1, const TB* B, int64_t sb0,
                 int64_t sb1, float* C, int64_t ldc, const float* bias, int relu, const float* mask, int64_t ldm,
                 int accumulate) {
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    k_gemm<TA, TB><<<grid, 256, 0, s>>>(M, N, K, A, sa0, sa1, B, sb0, sb1, C, ldc, bias, relu, mask, ldm, accumulate);
}

// dY = (Y - T) / n over the gathered rows; partial sums of squares per block
__global__ void k_mse(const float* __restrict__ Y, const float* __restrict__ T, const int* __restrict__ idx, int n,
                      int nout, float* __restrict__ dY, float* __restrict__ part) {
    __shared__ float red[256];
    float acc = 0.f;
    const float inv = 1.f / float(n);
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < (int64_t)n * nout; e += int64_t(gridDim.x) * blockDim.x) {
        const int i = int(e / nout), j = int(e % nout);
        const int src = idx ? idx[i] : i;
        const float r = Y[e] - T[(int64_t)src * nout + j];
        dY[e] = r * inv;
        acc += r * r;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_loss_finish(const float* __restrict__ part, int nb, int n, float* __restrict__ loss) {
    if (threadIdx.x != 0) return;
    double s = 0;
    for (int b = 0; b < nb; ++b) s += part[b];
    *loss = float(0.5 * s / n);
}

// db[j] = sum_i dY[i][j]: 64 columns per group, its 16 waves take every 16th row (each
// wave reads 64 consecutive floats of a row), then the 16 partial sums add through LDS
// in a fixed order
__global__ __launch_bounds__(1024) void k_colsum(const float* __restrict__ D, int n, int m, float* __restrict__ out) {
    __shared__ float red[16][64];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + l;
    float s = 0.f;
    if (j < m) {
#pragma unroll 8
        for (int i = w; i < n; i += 16) s += D[(int64_t)i * m + j];
    }
    red[w][l] = s;
    __syncthreads();
    if (w == 0 && j < m) {
        float t = 0.f;
        for (int k = 0; k < 16; ++k) t += red[k][l];
        out[j] = t;
    }
}

// gather rows: X[i] = src[idx[i]]
__global__ void k_gather_rows(const float* __restrict__ src, const int* __restrict__ idx, int n, int m,
                              float* __restrict__ dst) {
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < (int64_t)n * m; e += int64_t(gridDim.x) * blockDim.x)
        dst[e] = src[(int64_t)idx[e / m] * m + e % m];
}

// Adam on the FP32 master weights; refresh the bf16 copies of the matrices
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ g,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

__global__ void k_to_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = f2bf(src[i]);
}

__global__ void k_fill_int(int* __restrict__ p, int n) {
    if (threadIdx.x < n) p[threadIdx.x] = 0;
}

__global__ void k_zero_f(float* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) p[i] = 0.f;
}

// ---------------------------------------------------------------- leaf features and corrections
// s = ||r|| / sqrt(N) from a device norm; features of every leaf (cluster order)
// (halo block: the scaled means of the neighbour leaves listed in nbr, 6 values per slot)
__global__ void k_leaf_features(int nleaf, int n_pad, const int* __restrict__ lbeg, const int* __restrict__ lsize,
                                const int* __restrict__ perm, const double2* __restrict__ chi,
                                const double2* __restrict__ r, const double* __restrict__ norm, double sqrtN,
                                const int* __restrict__ nbr, int slots, const float* __restrict__ means,
                                float* __restrict__ X) {
    const int t = blockIdx.x;
    if (t >= nleaf) return;
    const int n = lsize[t], b = lbeg[t];
    double s = norm[0] / sqrtN;
    if (!(s > 0.0)) s = 1.0;
    const double inv = 1.0 / s;
    const int n_in = 7 * n_pad + 6 * slots;
    float* x = X + (int64_t)t * n_in;
    for (int e = 7 * n_pad + threadIdx.x; e < n_in; e += blockDim.x) {
        const int q = e - 7 * n_pad, nb = nbr[(int64_t)t * slots + q / 6];
        x[e] = nb >= 0 ? means[(int64_t)nb * 6 + q % 6] : 0.f;
    }
    for (int e = threadIdx.x; e < 7 * n_pad; e += blockDim.x) {
        float v = 0.f;
        if (e < 3 * n_pad) {
            const int i = e / 3, c = e % 3;
            if (i < n) v = float(r[(int64_t)perm[b + i] * 3 + c].x * inv);
        } else if (e < 6 * n_pad) {
            const int ee = e - 3 * n_pad, i = ee / 3, c = ee % 3;
            if (i < n) v = float(r[(int64_t)perm[b + i] * 3 + c].y * inv);
        } else {
            const int i = e - 6 * n_pad;
            if (i < n) v = float(chi[perm[b + i]].x);
        }
        x[e] = v;
    }
}

// Scaled leaf means [Re m_c, Im m_c] (c = 0..2) of r / s, one 64-lane group per leaf (leaves hold <= 64 voxels).
__global__ __launch_bounds__(64) void k_leaf_means(int nleaf, const int* __restrict__ lbeg, const int* __restrict__ lsize,
                                                   const int* __restrict__ perm, const double2* __restrict__ r,
                                                   const double* __restrict__ norm, double sqrtN, float* __restrict__ means) {
    __shared__ double red[6][64];
    const int t = blockIdx.x;
    if (t >= nleaf) return;                   // uniform over the group, before any barrier
    const int n = lsize[t], b = lbeg[t];
    const int i = threadIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (i < n) {
        const int64_t p = (int64_t)perm[b + i] * 3;
        for (int c = 0; c < 3; ++c) {
            const double2 a = r[p + c];
            v[c] = a.x;
            v[3 + c] = a.y;
        }
    }
    for (int q = 0; q < 6; ++q) red[q][i] = v[q];
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (i < w)
            for (int q = 0; q < 6; ++q) red[q][i] += red[q][i + w];
        __syncthreads();
    }
    if (i < 6) {
        double s = norm[0] / sqrtN;
        if (!(s > 0.0)) s = 1.0;
        means[(int64_t)t * 6 + i] = float(red[i][0] / (double(n) * s));
    }
}

// z (caller order) (+)= (Y_re + j Y_im) * s for every leaf
__global__ void k_leaf_scatter(int nleaf, int n_pad, const int* __restrict__ lbeg, const int* __restrict__ lsize,
                               const int* __restrict__ perm, const float* __restrict__ Y, const double* __restrict__ norm,
                               double sqrtN, double2* __restrict__ z, int accumulate) {
    const int t = blockIdx.x;
    if (t >= nleaf) return;
    const int n = lsize[t], b = lbeg[t];
    double s = norm[0] / sqrtN;
    if (!(s > 0.0)) s = 1.0;
    const float* y = Y + (int64_t)t * 6 * n_pad;
    for (int e = threadIdx.x; e < 3 * n; e += blockDim.x) {
        const int i = e / 3, c = e % 3;
        double2 v = make_double2(double(y[e]) * s, double(y[3 * n_pad + e]) * s);
        double2* out = z + (int64_t)perm[b + i] * 3 + c;
        if (accumulate) {
            const double2 o = *out;
            v.x += o.x;
            v.y += o.y;
        }
        *out = v;
    }
}

// targets [Re e_t, Im e_t] / s of every leaf
__global__ void k_leaf_targets(int nleaf, int n_pad, const int* __restrict__ lbeg, const int* __restrict__ lsize,
                               const int* __restrict__ perm, const double2* __restrict__ e, const double* __restrict__ norm,
                               double sqrtN, float* __restrict__ T) {
    const int t = blockIdx.x;
    if (t >= nleaf) return;
    const int n = lsize[t], b = lbeg[t];
    double s = norm[0] / sqrtN;
    if (!(s > 0.0)) s = 1.0;
    float* o = T + (int64_t)t * 6 * n_pad;
    for (int q = threadIdx.x; q < 6 * n_pad; q += blockDim.x) {
        float v = 0.f;
        const int part = q / (3 * n_pad), qq = q % (3 * n_pad), i = qq / 3, c = qq % 3;
        if (i < n) {
            const double2 a = e[(int64_t)perm[b + i] * 3 + c];
            v = float((part == 0 ? a.x : a.y) / s);
        }
        o[q] = v;
    }
}

__global__ void k_norm_full(const double2* __restrict__ a, int64_t N, double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0;
    for (int64_t i = threadIdx.x; i < N; i += 256) s += a[i].x * a[i].x + a[i].y * a[i].y;
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sqrt(red[0]);
}

// ---------------------------------------------------------------- block-diagonal fallback
// Inverse of M_t = I + alpha G_tt diag(chi_t) by Gauss-Jordan elimination with
// partial pivoting on the augmented matrix [M_t | I] (n x 2n, column major, kept
// in the preconditioner buffer; the inverse is its right half).  One group per leaf.
__global__ __launch_bounds__(256) void k_bd_setup(int nleaf, const int* __restrict__ lbeg, const int* __restrict__ lsize,
                                                  const int64_t* __restrict__ ldiag, const int* __restrict__ perm,
                                                  const double2* __restrict__ chi, const double2* __restrict__ near,
                                                  double alpha, const int64_t* __restrict__ loff,
                                                  double2* __restrict__ aug_all, int* __restrict__ singular) {
    __shared__ int piv;
    __shared__ double2 dinv_s;
    const int t = blockIdx.x;
    if (t >= nleaf) return;                   // uniform over the group, before any barrier
    const int n = lsize[t], b = lbeg[t];
    const double2* G = near + ldiag[t];
    double2* A = aug_all + loff[t];          // A(i, j) = A[i + j n], j < 2n
    for (int e = threadIdx.x; e < n * 2 * n; e += 256) {
        const int i = e % n, j = e / n;
        double2 v;
        if (j < n) {
            const double2 g = G[i + (int64_t)j * n];
            const double2 c = chi[perm[b + j]];
            v = make_double2(alpha * (g.x * c.x - g.y * c.y), alpha * (g.x * c.y + g.y * c.x));
            if (i == j) v.x += 1.0;
        } else {
            v = make_double2((j - n) == i ? 1.0 : 0.0, 0.0);
        }
        A[e] = v;
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (threadIdx.x == 0) {
            int p = k;
            double best = -1;
            for (int i = k; i < n; ++i) {
                const double2 a = A[i + (int64_t)k * n];
                const double m = a.x * a.x + a.y * a.y;
                if (m > best) { best = m; p = i; }
            }
            piv = p;
            if (best == 0.0) singular[0] = 1;
        }
        __syncthreads();
        const int p = piv;
        if (p != k)
            for (int j = threadIdx.x; j < 2 * n; j += 256) {
                const double2 tmp = A[k + (int64_t)j * n];
                A[k + (int64_t)j * n] = A[p + (int64_t)j * n];
                A[p + (int64_t)j * n] = tmp;
            }
        __syncthreads();
        if (threadIdx.x == 0) {
            const double2 d = A[k + (int64_t)k * n];
            const double den = d.x * d.x + d.y * d.y;
            dinv_s = den > 0 ? make_double2(d.x / den, -d.y / den) : make_double2(0, 0);
        }
        __syncthreads();
        const double2 dinv = dinv_s;
        for (int j = threadIdx.x; j < 2 * n; j += 256) {
            const double2 a = A[k + (int64_t)j * n];
            A[k + (int64_t)j * n] = make_double2(a.x * dinv.x - a.y * dinv.y, a.x * dinv.y + a.y * dinv.x);
        }
        __syncthreads();
        // eliminate column k from every other row; column k itself is cleared afterwards
        for (int e = threadIdx.x; e < n * 2 * n; e += 256) {
            const int i = e % n, j = e / n;
            if (i == k || j == k) continue;
            const double2 f = A[i + (int64_t)k * n];
            const double2 a = A[k + (int64_t)j * n];
            A[e] = make_double2(A[e].x - (f.x * a.x - f.y * a.y), A[e].y - (f.x * a.y + f.y * a.x));
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += 256)
            if (i != k) A[i + (int64_t)k * n] = make_double2(0, 0);
        __syncthreads();
    }
}

// z_t = inv_t r_t on each component (caller order)
__global__ __launch_bounds__(64) void k_bd_apply(int nleaf, const int* __restrict__ lbeg, const int* __restrict__ lsize,
                                                 const int* __restrict__ perm, const int64_t* __restrict__ loff,
                                                 const double2* __restrict__ inv, const double2* __restrict__ r,
                                                 double2* __restrict__ z) {
    __shared__ double2 rs[64 * 3];
    const int t = blockIdx.x;
    if (t >= nleaf) return;
    const int n = lsize[t], b = lbeg[t];
    for (int e = threadIdx.x; e < 3 * n; e += 64) rs[e] = r[(int64_t)perm[b + e / 3] * 3 + e % 3];
    __syncthreads();
    const int i = threadIdx.x;
    if (i >= n) return;
    const double2* Iv = inv + loff[t] + (int64_t)n * n;   // right half of [M | I] after elimination
    double2 a0 = make_double2(0, 0), a1 = a0, a2 = a0;
    for (int j = 0; j < n; ++j) {
        const double2 m = Iv[i + (int64_t)j * n];
        const double2 x0 = rs[j * 3], x1 = rs[j * 3 + 1], x2 = rs[j * 3 + 2];
        a0.x += m.x * x0.x - m.y * x0.y; a0.y += m.x * x0.y + m.y * x0.x;
        a1.x += m.x * x1.x - m.y * x1.y; a1.y += m.x * x1.y + m.y * x1.x;
        a2.x += m.x * x2.x - m.y * x2.y; a2.y += m.x * x2.y + m.y * x2.x;
    }
    const int64_t v = perm[b + i];
    z[v * 3] = a0;
    z[v * 3 + 1] = a1;
    z[v * 3 + 2] = a2;
}

// ---------------------------------------------------------------- MLP parameter layout
struct MlpLayout {
    int n_in, h, n_out;
    int64_t w1, b1, w2, b2, w3, b3, nmaster;   // float offsets in the master block
};

MlpLayout mlp_layout(int n_in, int h, int n_out) {
    MlpLayout L{};
    L.n_in = n_in;
    L.h = h;
    L.n_out = n_out;
    int64_t o = 0;
    L.w1 = o; o += int64_t(h) * n_in;
    L.b1 = o; o += h;
    L.w2 = o; o += int64_t(h) * h;
    L.b2 = o; o += h;
    L.w3 = o; o += int64_t(n_out) * h;
    L.b3 = o; o += n_out;
    L.nmaster = o;
    return L;
}

// params: [master f32][m f32][v f32][bf16 copy of master (all entries)]
struct MlpPtrs {
    float *master, *m, *v;
    uint16_t* bf;
};

static MlpPtrs mlp_ptrs(const MlpLayout& L, void* params) {
    MlpPtrs P;
    P.master = (float*)params;
    P.m = P.master + L.nmaster;
    P.v = P.m + L.nmaster;
    P.bf = (uint16_t*)(P.v + L.nmaster);
    return P;
}

size_t mlp_param_bytes(const MlpLayout& L) { return size_t(L.nmaster) * (12 + 2) + 256; }

// activations for a batch of n rows: H1, H2 (n x h), Y (n x n_out), dY, dH2, dH1, grads, partials, X/T gather
size_t mlp_work_bytes(const MlpLayout& L, int64_t n) {
    return size_t(n) * (2 * L.h + 2 * L.n_out + 2 * L.h + L.n_in + L.n_out) * 4 + size_t(L.nmaster) * 4 + 4096 * 4 + 1024;
}

struct MlpWork {
    float *H1, *H2, *Y, *dY, *dH2, *dH1, *Xg, *Tg, *grad, *part;
};

static MlpWork mlp_work(const MlpLayout& L, int64_t n, void* work) {
    MlpWork W;
    float* p = (float*)work;
    W.H1 = p; p += n * L.h;
    W.H2 = p; p += n * L.h;
    W.Y = p; p += n * L.n_out;
    W.dY = p; p += n * L.n_out;
    W.dH2 = p; p += n * L.h;
    W.dH1 = p; p += n * L.h;
    W.Xg = p; p += n * L.n_in;
    W.Tg = p; p += n * L.n_out;
    W.grad = p; p += L.nmaster;
    W.part = p;
    return W;
}

static int gridn(int64_t n) { return int(std::min<int64_t>((n + 255) / 256, 4096)); }

// Forward pass for rows X (n x n_in) -> Y (n x n_out) with bf16 weights.
void mlp_forward_dev(const MlpLayout& L, void* params, const float* X, float* H1, float* H2, float* Y, int64_t n,
                     hipStream_t s) {
    MlpPtrs P = mlp_ptrs(L, params);
    gemm<float, uint16_t>(s, int(n), L.h, L.n_in, X, L.n_in, 1, P.bf + L.w1, 1, L.n_in, H1, L.h, P.master + L.b1, 1,
                          nullptr, 0, 0);
    gemm<float, uint16_t>(s, int(n), L.h, L.h, H1, L.h, 1, P.bf + L.w2, 1, L.h, H2, L.h, P.master + L.b2, 1, nullptr, 0, 0);
    gemm<float, uint16_t>(s, int(n), L.n_out, L.h, H2, L.h, 1, P.bf + L.w3, 1, L.h, Y, L.n_out, P.master + L.b3, 0,
                          nullptr, 0, 0);
}

// Gradients of 0.5/n sum ||Y - T||^2 (rows idx of X, T, or all rows) into W.grad; loss into *loss.
void mlp_grad_dev(const MlpLayout& L, void* params, const float* X, const float* T, const int* idx, int64_t n,
                  MlpWork& W, float* loss, hipStream_t s) {
    MlpPtrs P = mlp_ptrs(L, params);
    const float* Xb = X;
    if (idx) {
        k_gather_rows<<<gridn(n * L.n_in), 256, 0, s>>>(X, idx, int(n), L.n_in, W.Xg);
        Xb = W.Xg;
    }
    mlp_forward_dev(L, params, Xb, W.H1, W.H2, W.Y, n, s);
    const int nb = gridn(n * L.n_out);
    k_mse<<<nb, 256, 0, s>>>(W.Y, T, idx, int(n), L.n_out, W.dY, W.part);
    if (loss) k_loss_finish<<<1, 64, 0, s>>>(W.part, nb, int(n), loss);
    float* g = W.grad;
    // layer 3: dW3 = dY^T H2, db3 = colsum dY
    gemm<float, float>(s, L.n_out, L.h, int(n), W.dY, 1, L.n_out, W.H2, L.h, 1, g + L.w3, L.h, nullptr, 0, nullptr, 0, 0);
    k_colsum<<<(L.n_out + 63) / 64, 1024, 0, s>>>(W.dY, int(n), L.n_out, g + L.b3);
    // dH2 = (dY W3) * (H2 > 0)
    gemm<float, uint16_t>(s, int(n), L.h, L.n_out, W.dY, L.n_out, 1, P.bf + L.w3, L.h, 1, W.dH2, L.h, nullptr, 0, W.H2,
                          L.h, 0);
    gemm<float, float>(s, L.h, L.h, int(n), W.dH2, 1, L.h, W.H1, L.h, 1, g + L.w2, L.h, nullptr, 0, nullptr, 0, 0);
    k_colsum<<<(L.h + 63) / 64, 1024, 0, s>>>(W.dH2, int(n), L.h, g + L.b2);
    // dH1 = (dH2 W2) * (H1 > 0)
    gemm<float, uint16_t>(s, int(n), L.h, L.h, W.dH2, L.h, 1, P.bf + L.w2, L.h, 1, W.dH1, L.h, nullptr, 0, W.H1, L.h, 0);
    gemm<float, float>(s, L.h, L.n_in, int(n), W.dH1, 1, L.h, Xb, L.n_in, 1, g + L.w1, L.n_in, nullptr, 0, nullptr, 0, 0);
    k_colsum<<<(L.h + 63) / 64, 1024, 0, s>>>(W.dH1, int(n), L.h, g + L.b1);
}

}  // namespace h2

using namespace h2;

extern "C" {

static h2_status mlp_check(const h2_mlp_dims* dm, MlpLayout* L) {
    if (!dm || dm->n_in < 1 || dm->n_hidden < 1 || dm->n_out < 1 || dm->n_in > 4096 || dm->n_hidden > 4096 ||
        dm->n_out > 4096)
        return handle_fail(H2_ERR_INVALID_ARG, "MLP sizes must be in [1, 4096]");
    *L = mlp_layout(dm->n_in, dm->n_hidden, dm->n_out);
    return H2_OK;
}

h2_status h2_mlp_sizes(const h2_mlp_dims* dm, int64_t batch, size_t* param_bytes, size_t* work_bytes) {
    MlpLayout L;
    h2_status st = mlp_check(dm, &L);
    if (st != H2_OK) return st;
    if (batch < 1) return handle_fail(H2_ERR_INVALID_ARG, "batch must be >= 1");
    if (param_bytes) *param_bytes = mlp_param_bytes(L);
    if (work_bytes) *work_bytes = mlp_work_bytes(L, batch);
    return H2_OK;
}

h2_status h2_mlp_set(const h2_mlp_dims* dm, void* params, const float* master_host, void* stream) {
    MlpLayout L;
    h2_status st = mlp_check(dm, &L);
    if (st != H2_OK) return st;
    if (!params || !master_host) return handle_fail(H2_ERR_INVALID_ARG, "null argument");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    MlpPtrs P = mlp_ptrs(L, params);
    if (hipMemcpyAsync(P.master, master_host, L.nmaster * 4, hipMemcpyHostToDevice, s) != hipSuccess)
        return handle_fail(H2_ERR_DEVICE, "upload failed");
    k_zero_f<<<gridn(2 * L.nmaster), 256, 0, s>>>(P.m, 2 * L.nmaster);
    k_to_bf16<<<gridn(L.nmaster), 256, 0, s>>>(P.master, P.bf, L.nmaster);
    if (hipStreamSynchronize(s) != hipSuccess) return handle_fail(H2_ERR_DEVICE, "synchronisation failed");
    return H2_OK;
}

h2_status h2_mlp_get(const h2_mlp_dims* dm, const void* params, float* master_host, void* stream) {
    MlpLayout L;
    h2_status st = mlp_check(dm, &L);
    if (st != H2_OK) return st;
    if (!params || !master_host) return handle_fail(H2_ERR_INVALID_ARG, "null argument");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(master_host, params, L.nmaster * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return handle_fail(H2_ERR_DEVICE, "download failed");
    return H2_OK;
}

h2_status h2_mlp_forward(const h2_mlp_dims* dm, void* params, const float* X, float* Y, int64_t n, void* work,
                         size_t work_bytes, void* stream) {
    MlpLayout L;
    h2_status st = mlp_check(dm, &L);
    if (st != H2_OK) return st;
    if (!params || !X || !Y || !work || n < 1) return handle_fail(H2_ERR_INVALID_ARG, "null argument or empty batch");
    if (work_bytes < mlp_work_bytes(L, n)) return handle_fail(H2_ERR_OOM, "MLP workspace too small");
    MlpWork W = mlp_work(L, n, work);
    mlp_forward_dev(L, params, X, W.H1, W.H2, Y, n, reinterpret_cast<hipStream_t>(stream));
    if (hipGetLastError() != hipSuccess) return handle_fail(H2_ERR_DEVICE, "MLP forward launch failed");
    return H2_OK;
}

h2_status h2_mlp_grad(const h2_mlp_dims* dm, void* params, const float* X, const float* T, int64_t n, float* grad,
                      float* loss, void* work, size_t work_bytes, void* stream) {
    MlpLayout L;
    h2_status st = mlp_check(dm, &L);
    if (st != H2_OK) return st;
    if (!params || !X || !T || !grad || !work || n < 1) return handle_fail(H2_ERR_INVALID_ARG, "null argument");
    if (work_bytes < mlp_work_bytes(L, n)) return handle_fail(H2_ERR_OOM, "MLP workspace too small");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    MlpWork W = mlp_work(L, n, work);
    mlp_grad_dev(L, params, X, T, nullptr, n, W, loss, s);
    if (hipMemcpyAsync(grad, W.grad, L.nmaster * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return handle_fail(H2_ERR_DEVICE, "copy failed");
    return H2_OK;
}

h2_status h2_mlp_train(const h2_mlp_dims* dm, void* params, const float* X, const float* T, int64_t n,
                       const int* order, int32_t epochs, int32_t batch, float lr, float* epoch_loss_host, void* work,
                       size_t work_bytes, void* stream) {
    MlpLayout L;
    h2_status st = mlp_check(dm, &L);
    if (st != H2_OK) return st;
    if (!params || !X || !T || !order || !work || n < 1 || epochs < 1 || batch < 1 || !(lr > 0))
        return handle_fail(H2_ERR_INVALID_ARG, "bad training arguments");
    if (work_bytes < mlp_work_bytes(L, batch)) return handle_fail(H2_ERR_OOM, "MLP workspace too small");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    MlpPtrs P = mlp_ptrs(L, params);
    MlpWork W = mlp_work(L, batch, work);
    float* dloss = W.part + 4096;
    int64_t step = 0;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    std::vector<float> hl;
    for (int ep = 0; ep < epochs; ++ep) {
        const int* ord = order + int64_t(ep) * n;
        double ep_loss = 0;
        int nb = 0;
        for (int64_t i0 = 0; i0 < n; i0 += batch) {
            const int64_t bn = std::min<int64_t>(batch, n - i0);
            mlp_grad_dev(L, params, X, T, ord + i0, bn, W, dloss, s);
            ++step;
            const float c1 = 1.f - std::pow(b1, float(step)), c2 = 1.f - std::pow(b2, float(step));
            k_adam<<<gridn(L.nmaster), 256, 0, s>>>(P.master, P.m, P.v, W.grad, L.nmaster, lr, b1, b2, eps, c1, c2);
            k_to_bf16<<<gridn(L.nmaster), 256, 0, s>>>(P.master, P.bf, L.nmaster);
            if (epoch_loss_host) {
                float lh = 0;
                if (hipMemcpyAsync(&lh, dloss, 4, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
                    return handle_fail(H2_ERR_DEVICE, "loss readback failed");
                ep_loss += lh;
                ++nb;
            }
        }
        if (epoch_loss_host) epoch_loss_host[ep] = float(ep_loss / std::max(nb, 1));
    }
    if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess)
        return handle_fail(H2_ERR_DEVICE, "training failed");
    return H2_OK;
}

}  // extern "C"

namespace h2 {

// device launch helpers used by h2vie_api.cpp and the solver
hipError_t launch_leaf_features(const LeafInfo& li, int n_pad, const int* perm, const double2* chi, const double2* r,
                                double* norm_scratch, int64_t N, const int* nbr, int slots, float* means, float* X,
                                hipStream_t s) {
    k_norm_full<<<1, 256, 0, s>>>(r, N, norm_scratch);
    if (slots > 0) k_leaf_means<<<li.n, 64, 0, s>>>(li.n, li.beg, li.size, perm, r, norm_scratch, std::sqrt(double(N)), means);
    k_leaf_features<<<li.n, 256, 0, s>>>(li.n, n_pad, li.beg, li.size, perm, chi, r, norm_scratch,
                                         std::sqrt(double(N)), nbr, slots, means, X);
    return hipGetLastError();
}

hipError_t launch_leaf_targets(const LeafInfo& li, int n_pad, const int* perm, const double2* e, const double* norm,
                               int64_t N, float* T, hipStream_t s) {
    k_leaf_targets<<<li.n, 256, 0, s>>>(li.n, n_pad, li.beg, li.size, perm, e, norm, std::sqrt(double(N)), T);
    return hipGetLastError();
}

hipError_t launch_leaf_scatter(const LeafInfo& li, int n_pad, const int* perm, const float* Y, const double* norm,
                               int64_t N, double2* z, int accumulate, hipStream_t s) {
    k_leaf_scatter<<<li.n, 256, 0, s>>>(li.n, n_pad, li.beg, li.size, perm, Y, norm, std::sqrt(double(N)), z,
                                        accumulate);
    return hipGetLastError();
}

hipError_t launch_bd_setup(const LeafInfo& li, const int* perm, const double2* chi, const double2* near, double alpha,
                           double2* inv, int* singular, hipStream_t s) {
    k_bd_setup<<<li.n, 256, 0, s>>>(li.n, li.beg, li.size, li.diag, perm, chi, near, alpha, li.inv_off, inv, singular);
    return hipGetLastError();
}

hipError_t launch_bd_apply(const LeafInfo& li, const int* perm, const double2* inv, const double2* r, double2* z,
                           hipStream_t s) {
    k_bd_apply<<<li.n, 64, 0, s>>>(li.n, li.beg, li.size, perm, li.inv_off, inv, r, z);
    return hipGetLastError();
}

hipError_t mlp_apply_handle(h2_handle h, const double2* r, double2* z, float* X, float* H1, float* H2, float* Y,
                            double* norm, hipStream_t s) {
    const DevH2& D = h->dev;
    const MlpLayout L = mlp_layout(h->mlp_dims.n_in, h->mlp_dims.n_hidden, h->mlp_dims.n_out);
    const int64_t N = int64_t(D.n_vox) * kNcomp;
    hipError_t e = launch_leaf_features(D.leaves, h->mlp_npad, D.perm, D.chi, r, norm, N, h->halo_nbr, h->halo_slots,
                                        h->halo_means, X, s);
    if (e != hipSuccess) return e;
    mlp_forward_dev(L, h->mlp_params, X, H1, H2, Y, D.leaves.n, s);
    const bool on_bd = h->mlp_base == H2_PRECOND_BLOCKDIAG;
    if (on_bd && (e = launch_bd_apply(D.leaves, D.perm, (const double2*)h->bd_buf, r, z, s)) != hipSuccess) return e;
    return launch_leaf_scatter(D.leaves, h->mlp_npad, D.perm, Y, norm, N, z, on_bd ? 1 : 0, s);
}

// X, H1, H2, Y for every leaf + one norm
size_t mlp_apply_work_bytes(h2_handle h) {
    const int64_t n = h->dev.leaves.n;
    const h2_mlp_dims& d = h->mlp_dims;
    return size_t(n) * (d.n_in + 2 * d.n_hidden + d.n_out) * 4 + 1024;
}

}  // namespace h2

extern "C" {

h2_status h2_leaf_count(h2_handle h, int32_t* n_leaves, int32_t* max_leaf) {
    if (!handle_live(h)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (n_leaves) *n_leaves = h->dev.leaves.n;
    if (max_leaf) *max_leaf = h->dev.leaves.max_leaf;
    return H2_OK;
}

h2_status h2_leaf_features(h2_handle h, int32_t n_pad, const void* r, float* X, void* scratch, void* stream) {
    if (!handle_live(h)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (!r || !X || !scratch) return handle_fail(H2_ERR_INVALID_ARG, "null argument");
    if (n_pad < h->dev.leaves.max_leaf || n_pad > 4096) return handle_fail(H2_ERR_INVALID_ARG, "n_pad below the largest leaf");
    const DevH2& D = h->dev;
    hipError_t e = launch_leaf_features(D.leaves, n_pad, D.perm, D.chi, (const double2*)r, (double*)scratch,
                                        int64_t(D.n_vox) * kNcomp, h->halo_nbr, h->halo_slots, h->halo_means, X,
                                        reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
    return H2_OK;
}

h2_status h2_leaf_targets(h2_handle h, int32_t n_pad, const void* ev, const void* r, float* T, void* scratch,
                          void* stream) {
    if (!handle_live(h)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (!ev || !r || !T || !scratch) return handle_fail(H2_ERR_INVALID_ARG, "null argument");
    if (n_pad < h->dev.leaves.max_leaf || n_pad > 4096) return handle_fail(H2_ERR_INVALID_ARG, "n_pad below the largest leaf");
    const DevH2& D = h->dev;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t N = int64_t(D.n_vox) * kNcomp;
    k_norm_full<<<1, 256, 0, s>>>((const double2*)r, N, (double*)scratch);
    hipError_t e = launch_leaf_targets(D.leaves, n_pad, D.perm, (const double2*)ev, (const double*)scratch, N, T, s);
    if (e != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
    return H2_OK;
}

h2_status h2_precond_blockdiag_bytes(h2_handle h, size_t* bytes) {
    if (!handle_live(h)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (!bytes) return handle_fail(H2_ERR_INVALID_ARG, "null argument");
    *bytes = size_t(h->dev.leaves.inv_elems) * 16 + 512;
    return H2_OK;
}

h2_status h2_precond_blockdiag(h2_handle h, void* buf, size_t bytes, void* stream) {
    if (!handle_live(h)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid handle");
    size_t need = 0;
    h2_precond_blockdiag_bytes(h, &need);
    if (!buf) return handle_fail(H2_ERR_INVALID_ARG, "null buffer");
    if (bytes < need) return handle_fail(H2_ERR_OOM, "block-diagonal buffer too small");
    if (reinterpret_cast<uintptr_t>(buf) % 256) return handle_fail(H2_ERR_INVALID_ARG, "buffer must be 256-byte aligned");
    const DevH2& D = h->dev;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int* flag = (int*)((char*)buf + size_t(D.leaves.inv_elems) * 16);
    k_fill_int<<<1, 64, 0, s>>>(flag, 1);
    hipError_t e = launch_bd_setup(D.leaves, D.perm, D.chi, (const double2*)D.tier[0].near, D.sigma * D.k * D.k * D.volume,
                                   (double2*)buf, flag, s);
    int hflag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
    if (hflag) return handle_fail(H2_ERR_INVALID_ARG, "a leaf diagonal block is singular");
    h->bd_buf = buf;
    h->bd_ready = true;
    return H2_OK;
}

h2_status h2_precond_mlp(h2_handle h, const h2_mlp_dims* dims, int32_t n_pad, void* params, int32_t base) {
    if (!handle_live(h)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid handle");
    MlpLayout L;
    h2_status st = mlp_check(dims, &L);
    if (st != H2_OK) return st;
    if (!params) return handle_fail(H2_ERR_INVALID_ARG, "null parameters");
    if (base != H2_PRECOND_NONE && base != H2_PRECOND_BLOCKDIAG)
        return handle_fail(H2_ERR_INVALID_ARG, "the MLP's base must be PRECOND_NONE or PRECOND_BLOCKDIAG");
    if (base == H2_PRECOND_BLOCKDIAG && !h->bd_ready)
        return handle_fail(H2_ERR_INVALID_ARG, "block-diagonal base not formed (h2_precond_blockdiag first)");
    if (n_pad < h->dev.leaves.max_leaf || dims->n_in != 7 * n_pad + 6 * h->halo_slots || dims->n_out != 6 * n_pad)
        return handle_fail(H2_ERR_INVALID_ARG,
                           "MLP sizes must be n_in = 7 n_pad + 6 halo slots, n_out = 6 n_pad, n_pad >= largest leaf");
    h->mlp_params = params;
    h->mlp_dims = *dims;
    h->mlp_npad = n_pad;
    h->mlp_base = base;
    return H2_OK;
}

h2_status h2_leaf_halo(h2_handle h, const int32_t* nbr, int32_t slots) {
    if (!handle_live(h)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (slots < 0 || slots > 124 || (slots > 0 && !nbr)) return handle_fail(H2_ERR_INVALID_ARG, "slots must be in [0, 124]");
    const int nl = h->dev.leaves.n;
    for (int64_t i = 0; i < int64_t(nl) * slots; ++i)
        if (nbr[i] < -1 || nbr[i] >= nl) return handle_fail(H2_ERR_INVALID_ARG, "neighbour index out of range");
    if (h->halo_nbr) (void)hipFree(h->halo_nbr);
    if (h->halo_means) (void)hipFree(h->halo_means);
    h->halo_nbr = nullptr;
    h->halo_means = nullptr;
    h->halo_slots = 0;
    h->mlp_params = nullptr;          // an attached MLP no longer matches the feature size
    if (slots == 0) return H2_OK;
    if (hipMalloc((void**)&h->halo_nbr, size_t(nl) * slots * 4) != hipSuccess ||
        hipMalloc((void**)&h->halo_means, size_t(nl) * 6 * 4) != hipSuccess)
        return handle_fail(H2_ERR_OOM, "halo tables: device allocation failed");
    if (hipMemcpy(h->halo_nbr, nbr, size_t(nl) * slots * 4, hipMemcpyHostToDevice) != hipSuccess)
        return handle_fail(H2_ERR_DEVICE, "halo table upload failed");
    h->halo_slots = slots;
    return H2_OK;
}

h2_status h2_precond_apply_bytes(h2_handle h, int32_t precond, size_t* bytes) {
    if (!handle_live(h)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (!bytes) return handle_fail(H2_ERR_INVALID_ARG, "null argument");
    if (precond == H2_PRECOND_MLP) {
        if (!h->mlp_params) return handle_fail(H2_ERR_INVALID_ARG, "no MLP attached");
        *bytes = mlp_apply_work_bytes(h) + 256;
    } else if (precond == H2_PRECOND_BLOCKDIAG) {
        *bytes = 0;
    } else {
        return handle_fail(H2_ERR_INVALID_ARG, "unknown preconditioner");
    }
    return H2_OK;
}

h2_status h2_precond_apply(h2_handle h, int32_t precond, const void* r, void* z, void* work, size_t work_bytes,
                           void* stream) {
    if (!handle_live(h)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid handle");
    size_t need = 0;
    h2_status st = h2_precond_apply_bytes(h, precond, &need);
    if (st != H2_OK) return st;
    if (!r || !z || r == z) return handle_fail(H2_ERR_INVALID_ARG, "r and z must be distinct device vectors");
    if (work_bytes < need || (need && !work)) return handle_fail(H2_ERR_OOM, "preconditioner workspace too small");
    const DevH2& D = h->dev;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e;
    if (precond == H2_PRECOND_BLOCKDIAG) {
        if (!h->bd_ready) return handle_fail(H2_ERR_INVALID_ARG, "block-diagonal preconditioner not formed");
        e = launch_bd_apply(D.leaves, D.perm, (const double2*)h->bd_buf, (const double2*)r, (double2*)z, s);
    } else {
        const h2_mlp_dims& dm = h->mlp_dims;
        const int64_t nl = D.leaves.n;
        char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(work) + 255) & ~uintptr_t(255));
        float* X = (float*)base;
        float* H1 = X + nl * dm.n_in;
        float* H2 = H1 + nl * dm.n_hidden;
        float* Y = H2 + nl * dm.n_hidden;
        double* nrm = (double*)(Y + nl * dm.n_out + 2);     // 8-byte aligned: every block above is a float count * 4
        nrm = (double*)((reinterpret_cast<uintptr_t>(nrm) + 7) & ~uintptr_t(7));
        e = mlp_apply_handle(h, (const double2*)r, (double2*)z, X, H1, H2, Y, nrm, s);
    }
    if (e != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
    return H2_OK;
}

}  // extern "C"
