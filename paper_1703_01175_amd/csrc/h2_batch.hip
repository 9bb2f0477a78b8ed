// Batched BF16x3 tier kernels: operand packing, bf16 hi/lo splits and the
// block GEMM on the matrix cores (v_mfma_f32_16x16x32_bf16).
//
// Lane layout of the 16x16x32 bf16 MFMA (checked on gfx950): lane l holds
// A[l % 16][8 (l / 16) + q] and B[8 (l / 16) + q][l % 16] for q = 0..7, and the
// result C[4 (l / 16) + r][l % 16] for r = 0..3.
#include <hip/hip_runtime.h>

#include "h2_batch.h"
#include "h2_internal.h"

namespace h2 {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_val(uint32_t b) { return __uint_as_float(b << 16); }

// hi = bf16(v), lo = bf16(v - hi)
__device__ __forceinline__ void split2(float v, uint16_t& hi, uint16_t& lo) {
    uint32_t h = bf16_bits(v);
    hi = (uint16_t)h;
    lo = (uint16_t)bf16_bits(v - bf16_val(h));
}

// ---------------------------------------------------------------- packing
// One 256-thread group per job: A(i, k) for i < mp, k < kp (zero padded).
__global__ __launch_bounds__(256) void k_pack(const PackJob* __restrict__ jobs, const double2* __restrict__ s0,
                                              const double2* __restrict__ s1, const double2* __restrict__ s2,
                                              const double2* __restrict__ s3, uint16_t* __restrict__ arena) {
    const PackJob J = jobs[blockIdx.x];
    const double2* src = J.which == 0 ? s0 : J.which == 1 ? s1 : J.which == 2 ? s2 : s3;
    src += J.src;
    const int64_t plane = int64_t(J.mp) * J.kp;
    uint16_t* d = arena + J.dst;
    for (int e = threadIdx.x; e < J.mp * J.kp; e += 256) {
        const int i = e / J.kp, k = e % J.kp;
        double2 v = make_double2(0, 0);
        if (i < J.m && k < J.k) v = J.transpose ? src[k + (int64_t)i * J.src_rows] : src[i + (int64_t)k * J.src_rows];
        uint16_t rh, rl, ih, il;
        split2((float)v.x, rh, rl);
        split2((float)v.y, ih, il);
        d[e] = rh;
        d[plane + e] = rl;
        d[2 * plane + e] = ih;
        d[3 * plane + e] = il;
    }
}

__global__ void k_fill_u16(uint16_t* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) p[i] = 0;
}

// ---------------------------------------------------------------- vectors
// U planes: column j = 3 r + c, row prow[p]: chi[v] x[3 v + c + r ldx] (op Z) or x (op G)
__global__ void k_prologue_b(int n_vox, const int* __restrict__ perm, const int* __restrict__ prow,
                             const double2* __restrict__ chi, const float2* __restrict__ x, int64_t ldx, int ncols,
                             uint16_t* __restrict__ Ub, int64_t urows, int64_t plane, int op) {
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < (int64_t)n_vox * ncols;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int p = int(e % n_vox);
        const int j = int(e / n_vox);
        const int v = perm[p];
        const int r = j / 3, c = j % 3;
        float2 a = x[(int64_t)v * 3 + c + r * ldx];
        float re = a.x, im = a.y;
        if (op == 1) {
            const float cr = (float)chi[v].x, ci = (float)chi[v].y;
            re = cr * a.x - ci * a.y;
            im = cr * a.y + ci * a.x;
        }
        const int64_t o = (int64_t)j * urows + prow[p];
        uint16_t h, l;
        split2(re, h, l);
        Ub[o] = h;
        Ub[plane + o] = l;
        split2(im, h, l);
        Ub[2 * plane + o] = h;
        Ub[3 * plane + o] = l;
    }
}

// y[3 v + c + r ldy] = x + alpha Y (op Z) or Y (op G), Y from FP32 planes
__global__ void k_epilogue_b(int n_vox, const int* __restrict__ perm, const int* __restrict__ prow,
                             const float* __restrict__ Yf, int64_t urows, int64_t plane, const float2* __restrict__ x,
                             int64_t ldx, float2* __restrict__ y, int64_t ldy, int ncols, int op, float alpha) {
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < (int64_t)n_vox * ncols;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int p = int(e % n_vox);
        const int j = int(e / n_vox);
        const int v = perm[p];
        const int r = j / 3, c = j % 3;
        const int64_t o = (int64_t)j * urows + prow[p];
        float re = Yf[o], im = Yf[plane + o];
        if (op == 1) {
            const float2 a = x[(int64_t)v * 3 + c + r * ldx];
            re = a.x + alpha * re;
            im = a.y + alpha * im;
        }
        y[(int64_t)v * 3 + c + r * ldy] = make_float2(re, im);
    }
}

// FP32 planes -> bf16 hi/lo planes for rows [r0, r0 + nrows) of every column.
__global__ void k_split(const SplitSeg* __restrict__ segs, const int* __restrict__ seg_cols) {
    const SplitSeg S = segs[blockIdx.y];
    const int ncols = seg_cols[blockIdx.y];
    const int64_t n = (int64_t)S.nrows * ncols;
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t row = S.r0 + e % S.nrows;
        const int64_t col = e / S.nrows;
        const float re = S.src[col * S.sld + row], im = S.src[S.sps + col * S.sld + row];
        const int64_t o = col * S.dld + row;
        uint16_t h, l;
        split2(re, h, l);
        S.dst[o] = h;
        S.dst[S.dps + o] = l;
        split2(im, h, l);
        S.dst[2 * S.dps + o] = h;
        S.dst[3 * S.dps + o] = l;
    }
}

// ---------------------------------------------------------------- block GEMM
union V8 {
    uint4 u;
    bf16x8 b;
};

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {
    V8 v;
    v.u = *reinterpret_cast<const uint4*>(p);
    return v.b;
}
__device__ __forceinline__ bf16x8 ld8_neg(const uint16_t* p, bool neg) {
    V8 v;
    v.u = *reinterpret_cast<const uint4*>(p);
    if (neg) {
        v.u.x ^= 0x80008000u;
        v.u.y ^= 0x80008000u;
        v.u.z ^= 0x80008000u;
        v.u.w ^= 0x80008000u;
    }
    return v.b;
}
__device__ __forceinline__ bf16x8 zero8() {
    V8 v;
    v.u = make_uint4(0, 0, 0, 0);
    return v.b;
}

__device__ __forceinline__ bf16x8 lds8(const uint16_t* p) {
    V8 v;
    v.u = *reinterpret_cast<const uint4*>(p);
    return v.b;
}

// One group per task (owner, first column); wave w owns real row tiles w and w + 4
// of the owner (2 mp real rows) and all NC / 16 column tiles of the task.  The B
// operand of each term (the source's rows of the task's columns, re and im, hi and
// lo) is staged once in LDS and read from there by all four waves; each wave reads
// its own rows of A straight from memory (A is used once per task).
template <int NC>
__global__ __launch_bounds__(256) void k_bgemm(const BOwner* __restrict__ owners, const BTerm* __restrict__ terms,
                                               const int2* __restrict__ tasks, const int* __restrict__ owner_cols) {
    constexpr int NCT = NC / 16;
    constexpr int BST = 2 * 64 + 8;   // LDS column stride (bf16): 2 kp <= 128 real k, padded against bank conflicts
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][NC * BST];   // [hi, lo][column][re k | im k]
    const int2 task = tasks[blockIdx.x];
    const BOwner O = owners[task.x];
    const int ncols = owner_cols[task.x];
    const int col0 = task.y;
    const int nc_here = min(NC, ncols - col0);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    const int mp = O.mp;
    const int nrt = (2 * mp) / 16;
    const bool v0 = w < nrt, v1 = (w + 4) < nrt;   // waves without a row tile still stage B
    f32x4 acc[2][NCT];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < NCT; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    // rows of my tiles: real row rr = rt * 16 + l % 16 -> half h, complex row i
    int hrow[2], irow[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int rr = (w + 4 * r) * 16 + (l & 15);
        hrow[r] = rr >= mp;
        irow[r] = rr - hrow[r] * mp;
    }
    for (int t = O.t0; t < O.t0 + O.nt; ++t) {
        const BTerm T = terms[t];
        const int kp = T.kp;
        const int kq = kp >> 3;                       // 16-byte chunks per plane column
        __syncthreads();                              // the previous term's B is no longer read
        for (int e = threadIdx.x; e < NC * 4 * kq; e += 256) {
            const int c = e / (4 * kq);
            const int rem = e - c * 4 * kq;
            const int plane = rem / kq, kc = rem - plane * kq;   // plane: re_hi, re_lo, im_hi, im_lo
            uint4 v = make_uint4(0, 0, 0, 0);
            if (c < nc_here)
                v = *reinterpret_cast<const uint4*>(T.b + plane * T.bps + (int64_t)(col0 + c) * T.bld + kc * 8);
            *reinterpret_cast<uint4*>(&Bs[plane & 1][c * BST + (plane >> 1) * kp + kc * 8]) = v;
        }
        __syncthreads();
        if (!v0) continue;
        const int64_t pl = (int64_t)mp * kp;
        const int nks = (2 * kp) / 32;
        for (int ks = 0; ks < nks; ++ks) {
            const int kreal = ks * 32 + 8 * (l >> 4);
            const int kh = kreal >= kp;
            const int kk = kreal - kh * kp;
            bf16x8 ahi[2], alo[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                if (r == 0 || v1) {
                    const int h = hrow[r];
                    const bool use_im = (h != kh);                 // [Ar -Ai; Ai Ar]
                    const bool neg = (h == 0) && (kh == 1);
                    const uint16_t* pa = T.a + (use_im ? 2 * pl : 0) + (int64_t)irow[r] * kp + kk;
                    ahi[r] = ld8_neg(pa, neg);
                    alo[r] = ld8_neg(pa + pl, neg);
                } else {
                    ahi[r] = zero8();
                    alo[r] = zero8();
                }
            }
#pragma unroll
            for (int c = 0; c < NCT; ++c) {
                const uint16_t* pb = &Bs[0][(c * 16 + (l & 15)) * BST + kreal];
                const bf16x8 bhi = lds8(pb), blo = lds8(pb + NC * BST);
                acc[0][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[0], bhi, acc[0][c], 0, 0, 0);
                acc[0][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[0], blo, acc[0][c], 0, 0, 0);
                acc[0][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[0], bhi, acc[0][c], 0, 0, 0);
                if (v1) {
                    acc[1][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[1], bhi, acc[1][c], 0, 0, 0);
                    acc[1][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[1], blo, acc[1][c], 0, 0, 0);
                    acc[1][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[1], bhi, acc[1][c], 0, 0, 0);
                }
            }
        }
    }
    if (!v0) return;
    // lane holds C[4 (l / 16) + q][l % 16] of each tile: 4 consecutive rows of one column
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        if (r == 1 && !v1) break;
        const int rr0 = (w + 4 * r) * 16 + 4 * (l >> 4);
        const int h = rr0 >= mp;
        const int i0 = rr0 - h * mp;
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
            const int col = col0 + c * 16 + (l & 15);
            if (col >= ncols) continue;
            float4* dst = reinterpret_cast<float4*>(O.out + h * O.ps + (int64_t)col * O.ld + i0);
            float4 v = make_float4(acc[r][c][0], acc[r][c][1], acc[r][c][2], acc[r][c][3]);
            if (O.acc) {
                const float4 o = *dst;
                v.x += o.x; v.y += o.y; v.z += o.z; v.w += o.w;
            }
            *dst = v;
        }
    }
}

static int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    return int(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

hipError_t launch_pack(const PackJob* jobs_dev, int njobs, const double2* const* srcs, uint16_t* arena,
                       hipStream_t s) {
    if (njobs == 0) return hipSuccess;
    // grid.x limit is far above the job counts here (one group per block)
    k_pack<<<njobs, 256, 0, s>>>(jobs_dev, srcs[0], srcs[1], srcs[2], srcs[3], arena);
    return hipGetLastError();
}

hipError_t launch_fill_u16(uint16_t* p, int64_t n, hipStream_t s) {
    k_fill_u16<<<grid_for(n), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_prologue_b(int n_vox, const int* perm, const int* prow, const double2* chi, const float2* x,
                             int64_t ldx, int ncols, uint16_t* Ub, int64_t urows, int64_t plane, int op, hipStream_t s) {
    k_prologue_b<<<grid_for((int64_t)n_vox * ncols), 256, 0, s>>>(n_vox, perm, prow, chi, x, ldx, ncols, Ub, urows,
                                                                  plane, op);
    return hipGetLastError();
}

hipError_t launch_epilogue_b(int n_vox, const int* perm, const int* prow, const float* Yf, int64_t urows,
                             int64_t plane, const float2* x, int64_t ldx, float2* y, int64_t ldy, int ncols, int op,
                             float alpha, hipStream_t s) {
    k_epilogue_b<<<grid_for((int64_t)n_vox * ncols), 256, 0, s>>>(n_vox, perm, prow, Yf, urows, plane, x, ldx, y, ldy,
                                                                  ncols, op, alpha);
    return hipGetLastError();
}

hipError_t launch_split(const SplitSeg* segs, int nseg, int max_elems_per_seg, const int* seg_cols, hipStream_t s) {
    if (nseg == 0) return hipSuccess;
    dim3 grid(grid_for(max_elems_per_seg) > 2048 ? 2048 : grid_for(max_elems_per_seg), nseg);
    k_split<<<grid, 256, 0, s>>>(segs, seg_cols);
    return hipGetLastError();
}

hipError_t launch_bgemm(int nc, const BOwner* owners, const BTerm* terms, const int2* tasks, int ntasks,
                        const int* owner_cols, hipStream_t s) {
    if (ntasks == 0) return hipSuccess;
    if (nc == 32)
        k_bgemm<32><<<ntasks, 256, 0, s>>>(owners, terms, tasks, owner_cols);
    else if (nc == 64)
        k_bgemm<64><<<ntasks, 256, 0, s>>>(owners, terms, tasks, owner_cols);
    else if (nc == 128)
        k_bgemm<128><<<ntasks, 256, 0, s>>>(owners, terms, tasks, owner_cols);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace h2
