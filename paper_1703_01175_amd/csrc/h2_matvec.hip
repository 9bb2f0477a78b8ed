// H^2 matrix-vector product on gfx950 (Sec. IV.B of Omar & Jiao).
//
//   prologue      U = chi . x, permuted into tree order        (kappa(r') of eq. (1))
//   leaf forward  X_t = V_t^T U_t                              (forward transformation)
//   upward        X_p = sum_c T_c^T X_c, level by level         (nested bases, eq. (9))
//   coupling      Y_t = sum_{s in R_t} S_ts X_s, all levels     (coupling multiplication)
//   downward      Y_c += T_c Y_p, level by level                (backward transformation)
//   near+leaf     y_t = sum_s G_ts U_s + V_t Y_t, then z = x + sigma k^2 V y (epilogue)
//
// Plain transposes (not conjugates) throughout, as the paper's transforms use
// (V^s)^T.  Every kernel is templated on the block storage type TB and the
// vector/accumulation type TV (double2 for FP64, float2 for FP32).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "h2_internal.h"

namespace h2 {

template <typename TV> struct Real;
template <> struct Real<double2> { using T = double; };
template <> struct Real<float2> { using T = float; };

template <typename TV, typename TB>
__device__ __forceinline__ void cfma(TV& acc, TB a, TV b) {
    using R = typename Real<TV>::T;
    R ax = (R)a.x, ay = (R)a.y;
    acc.x = fma(ax, b.x, acc.x);
    acc.x = fma(-ay, b.y, acc.x);
    acc.y = fma(ax, b.y, acc.y);
    acc.y = fma(ay, b.x, acc.y);
}

template <typename TV> __device__ __forceinline__ TV czero() { TV z; z.x = 0; z.y = 0; return z; }

// FP64 matrix-core product D = A B + C on 16 x 16 x 4 tiles (one double of A and of B
// per lane, four of D).
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Streaming (nontemporal) loads of block data: read once per product, kept out
// of the caches that hold the reused vectors.
__device__ __forceinline__ double2 ldnt(const double2* p) {
    return make_double2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}
__device__ __forceinline__ float2 ldnt(const float2* p) {
    return make_float2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}

// Near-block loads: streaming (nontemporal) when every block is read once per
// product, plain cached loads when identical blocks are stored once and reread.
template <bool NT, typename T> __device__ __forceinline__ T ldblk(const T* p) {
    if constexpr (NT) return ldnt(p);
    else return *p;
}

// Broadcast lane J of each 16-lane row to the whole row (DPP row_newbcast).
template <int J> __device__ __forceinline__ double bcast_row(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, 0x150 + J, 0xf, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, 0x150 + J, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
template <int J> __device__ __forceinline__ float bcast_row(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x150 + J, 0xf, 0xf, false));
}
template <int J, typename TV> __device__ __forceinline__ TV bcast_row2(TV v) {
    TV r;
    r.x = bcast_row<J>(v.x);
    r.y = bcast_row<J>(v.y);
    return r;
}

template <typename TV>
__device__ __forceinline__ TV cadd(TV a, TV b) { TV r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }

// ---------------------------------------------------------------- prologue
// U[p][c] = chi[perm[p]] * x[3 perm[p] + c]  (op Z)   or   x[3 perm[p] + c]  (op G)
template <typename TV>
__global__ void k_prologue(int n_vox, const int* __restrict__ perm, const double2* __restrict__ chi,
                           const TV* __restrict__ x, TV* __restrict__ U, int op) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_vox) return;
    int v = perm[p];
    using R = typename Real<TV>::T;
    TV c;
    if (op == 1) { c.x = (R)chi[v].x; c.y = (R)chi[v].y; } else { c.x = 1; c.y = 0; }
#pragma unroll
    for (int q = 0; q < kNcomp; ++q) {
        TV a = x[(int64_t)v * kNcomp + q];
        TV r;
        r.x = c.x * a.x - c.y * a.y;
        r.y = c.x * a.y + c.y * a.x;
        U[(int64_t)p * kNcomp + q] = r;
    }
}

// ---------------------------------------------------------------- leaf forward
// X_t[a][c] = sum_i V_t[i, a] U_t[i][c]; one 64-thread group per leaf.
template <typename TB, typename TV>
__global__ __launch_bounds__(64) void k_leaf_forward(const int* __restrict__ leaf_id, const int* __restrict__ cl_rank,
                                                     const int* __restrict__ cl_coef, const int* __restrict__ cl_begin,
                                                     const int* __restrict__ cl_size, const int64_t* __restrict__ cl_basis_off,
                                                     const TB* __restrict__ basis, const TV* __restrict__ U,
                                                     TV* __restrict__ Xh) {
    __shared__ TV su[kMaxLeaf * kNcomp];
    const int t = leaf_id[blockIdx.x];
    const int k = cl_rank[t];
    if (k == 0) return;
    const int n = cl_size[t];
    const int b0 = cl_begin[t];
    for (int e = threadIdx.x; e < n * kNcomp; e += 64) su[e] = U[(int64_t)b0 * kNcomp + e];
    __syncthreads();
    const TB* V = basis + cl_basis_off[t];
    const int co = cl_coef[t];
    for (int a = threadIdx.x; a < k; a += 64) {
        TV acc0 = czero<TV>(), acc1 = czero<TV>(), acc2 = czero<TV>();
        const TB* col = V + (int64_t)a * n;
        // unrolled so that several loads are in flight (the loop is latency-bound)
#pragma unroll 8
        for (int i = 0; i < n; ++i) {
            TB v = col[i];
            cfma(acc0, v, su[i * 3 + 0]);
            cfma(acc1, v, su[i * 3 + 1]);
            cfma(acc2, v, su[i * 3 + 2]);
        }
        TV* o = Xh + (int64_t)(co + a) * kNcomp;
        o[0] = acc0; o[1] = acc1; o[2] = acc2;
    }
}

// ---------------------------------------------------------------- upward pass
// X_p[a][c] = sum_children sum_b T_c[b, a] X_c[b][c]
template <typename TB, typename TV>
__global__ __launch_bounds__(64) void k_transfer_up(const int* __restrict__ list, const int* __restrict__ cl_rank,
                                                    const int* __restrict__ cl_coef, const int* __restrict__ cl_first_child,
                                                    const int* __restrict__ cl_nchild, const int64_t* __restrict__ cl_toff,
                                                    const TB* __restrict__ transfer, TV* __restrict__ Xh) {
    const int p = list[blockIdx.x];
    const int kp = cl_rank[p];
    const int c0 = cl_first_child[p], nc = cl_nchild[p];
    for (int a = threadIdx.x; a < kp; a += 64) {
        TV acc0 = czero<TV>(), acc1 = czero<TV>(), acc2 = czero<TV>();
        for (int ch = c0; ch < c0 + nc; ++ch) {
            const int kc = cl_rank[ch];
            if (kc == 0) continue;
            const TB* T = transfer + cl_toff[ch] + (int64_t)a * kc;
            const TV* xc = Xh + (int64_t)cl_coef[ch] * kNcomp;
#pragma unroll 8
            for (int b = 0; b < kc; ++b) {
                TB tv = T[b];
                cfma(acc0, tv, xc[b * 3 + 0]);
                cfma(acc1, tv, xc[b * 3 + 1]);
                cfma(acc2, tv, xc[b * 3 + 2]);
            }
        }
        TV* o = Xh + (int64_t)(cl_coef[p] + a) * kNcomp;
        o[0] = acc0; o[1] = acc1; o[2] = acc2;
    }
}

// ---------------------------------------------------------------- couplings
// Y_t = [S_ts1 S_ts2 ...] * gather(X_s): the grouped block row of t (k_t x ncols,
// column major) times the gathered coefficients.  A wave is G = 64/R column
// groups of R row lanes (R = 16, 32 or 64 by rank).  Per super-step of 16*G
// columns, lane i of every 16-lane DPP row fetches the coefficients of one
// column (column base + G*i + g of its group g), and step j broadcasts lane j's
// coefficients across the row while every lane streams S(row, base + G*j + g):
// each load instruction covers G consecutive columns of the column-major block.
template <int J, typename TB, typename TV>
__device__ __forceinline__ void coup_step(const TB* sv, TV x0, TV x1, TV x2, TV& a0, TV& a1, TV& a2) {
    TV b0 = bcast_row2<J>(x0), b1 = bcast_row2<J>(x1), b2 = bcast_row2<J>(x2);
    cfma(a0, sv[J], b0);
    cfma(a1, sv[J], b1);
    cfma(a2, sv[J], b2);
}

template <typename TB, typename TV, int R>
__device__ __forceinline__ void coupling_rows(int kt, int ncols, const TB* __restrict__ S, const int* __restrict__ src,
                                              const TV* __restrict__ Xh, TV* __restrict__ Yh, int co, TV* red) {
    constexpr int G = 64 / R;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int a = lane % R;
    const int g = lane / R;
    const int i16 = lane & 15;
    for (int r0 = 0; r0 < kt; r0 += R) {
        const int row = r0 + a;
        const bool live = row < kt;
        TV acc0 = czero<TV>(), acc1 = czero<TV>(), acc2 = czero<TV>();
        for (int base = w * 16 * G; base < ncols; base += 4 * 16 * G) {
            const int cx = base + G * i16 + g;
            TV x0 = czero<TV>(), x1 = czero<TV>(), x2 = czero<TV>();
            if (cx < ncols) {
                const TV* xs = Xh + (int64_t)src[cx] * kNcomp;
                x0 = xs[0];
                x1 = xs[1];
                x2 = xs[2];
            }
            TB sv[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int c = base + G * q + g;
                if (live && c < ncols) sv[q] = ldnt(S + (int64_t)c * kt + row);
                else { sv[q].x = 0; sv[q].y = 0; }
            }
            coup_step<0>(sv, x0, x1, x2, acc0, acc1, acc2);
            coup_step<1>(sv, x0, x1, x2, acc0, acc1, acc2);
            coup_step<2>(sv, x0, x1, x2, acc0, acc1, acc2);
            coup_step<3>(sv, x0, x1, x2, acc0, acc1, acc2);
            coup_step<4>(sv, x0, x1, x2, acc0, acc1, acc2);
            coup_step<5>(sv, x0, x1, x2, acc0, acc1, acc2);
            coup_step<6>(sv, x0, x1, x2, acc0, acc1, acc2);
            coup_step<7>(sv, x0, x1, x2, acc0, acc1, acc2);
            coup_step<8>(sv, x0, x1, x2, acc0, acc1, acc2);
            coup_step<9>(sv, x0, x1, x2, acc0, acc1, acc2);
            coup_step<10>(sv, x0, x1, x2, acc0, acc1, acc2);
            coup_step<11>(sv, x0, x1, x2, acc0, acc1, acc2);
            coup_step<12>(sv, x0, x1, x2, acc0, acc1, acc2);
            coup_step<13>(sv, x0, x1, x2, acc0, acc1, acc2);
            coup_step<14>(sv, x0, x1, x2, acc0, acc1, acc2);
            coup_step<15>(sv, x0, x1, x2, acc0, acc1, acc2);
        }
        // threadIdx.x = w*64 + g*R + a: reduce over the 4 waves and G groups of each row
        red[threadIdx.x * 3 + 0] = acc0;
        red[threadIdx.x * 3 + 1] = acc1;
        red[threadIdx.x * 3 + 2] = acc2;
        __syncthreads();
        if (threadIdx.x < R * 3) {
            const int aa = threadIdx.x / 3, q = threadIdx.x % 3;
            TV sum = czero<TV>();
#pragma unroll
            for (int ww = 0; ww < 4; ++ww)
#pragma unroll
                for (int gg = 0; gg < G; ++gg) sum = cadd(sum, red[(ww * 64 + gg * R + aa) * 3 + q]);
            if (r0 + aa < kt) Yh[(int64_t)(co + r0 + aa) * kNcomp + q] = sum;
        }
        __syncthreads();
    }
}

template <typename TB, typename TV>
__global__ __launch_bounds__(256) void k_coupling(const int* __restrict__ row_cl, const int* __restrict__ row_ncols,
                                                  const int64_t* __restrict__ row_off, const int* __restrict__ row_colptr,
                                                  const int* __restrict__ colsrc, const int* __restrict__ cl_rank,
                                                  const int* __restrict__ cl_coef, const TB* __restrict__ coupling,
                                                  const TV* __restrict__ Xh, TV* __restrict__ Yh) {
    __shared__ TV red[256 * 3];
    const int slot = blockIdx.x;
    const int t = row_cl[slot];
    const int kt = cl_rank[t];
    const int ncols = row_ncols[slot];
    const TB* S = coupling + row_off[slot];
    const int* src = colsrc + row_colptr[slot];
    const int co = cl_coef[t];
    if (kt <= 16)
        coupling_rows<TB, TV, 16>(kt, ncols, S, src, Xh, Yh, co, red);
    else if (kt <= 32)
        coupling_rows<TB, TV, 32>(kt, ncols, S, src, Xh, Yh, co, red);
    else
        coupling_rows<TB, TV, 64>(kt, ncols, S, src, Xh, Yh, co, red);
}

// ---------------------------------------------------------------- symmetric couplings
// Row slot t streams only the blocks it owns (one of each unordered admissible pair
// {t, s}; S_st = S_ts^T) and applies each twice: Y_t += S_ts X_s, and the column
// sums S_ts^T X_t (3 complex per owned column) go to `part` for cluster s, which
// adds them in k_coupling_recv.  Lanes: RL row lanes per column (RL = 4, 8, 16 for
// k_t <= 16, 32, 64), 64 / RL columns per wave step; lane (cg, rl) holds rows
// rl + RL q (q < 4) of its column, so each column's transposed sum is a butterfly
// over RL neighbouring lanes, and the lane's X_t rows stay in registers.

// DPP move of a double / float within 16-lane rows
template <int CTRL> __device__ __forceinline__ double dpp_mov(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL> __device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL, typename TV> __device__ __forceinline__ TV dpp_add(TV v) {
    TV r;
    r.x = v.x + dpp_mov<CTRL>(v.x);
    r.y = v.y + dpp_mov<CTRL>(v.y);
    return r;
}
constexpr int kDppXor1 = 0xB1;       // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;       // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;
constexpr int kDppRor4 = 0x124;
constexpr int kDppRor8 = 0x128;

// Lane exchange across 16-lane rows (ds_bpermute on 32-bit halves).
__device__ __forceinline__ double shfl_xor_r(double v, int m) {
    const int lane = threadIdx.x & 63;
    const int src = ((lane ^ m) & 63) << 2;
    const int lo = __builtin_amdgcn_ds_bpermute(src, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(src, __double2hiint(v));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float shfl_xor_r(float v, int m) {
    const int lane = threadIdx.x & 63;
    return __int_as_float(__builtin_amdgcn_ds_bpermute(((lane ^ m) & 63) << 2, __float_as_int(v)));
}

// Sum over the RL neighbouring lanes of a column (butterfly; every lane gets the sum).
template <int RL, typename TV> __device__ __forceinline__ TV col_sum(TV v) {
    v = dpp_add<kDppXor1>(v);
    v = dpp_add<kDppXor2>(v);
    if constexpr (RL >= 8) v = dpp_add<kDppHalfMirror>(v);
    if constexpr (RL >= 16) v = dpp_add<kDppMirror>(v);
    return v;
}

template <int C, typename TV> __device__ __forceinline__ TV quad_bcast(TV v) {
    constexpr int ctrl = C | (C << 2) | (C << 4) | (C << 6);     // quad_perm [C, C, C, C]
    TV r;
    r.x = dpp_mov<ctrl>(v.x);
    r.y = dpp_mov<ctrl>(v.y);
    return r;
}

// An integer zero the compiler cannot see through: LDS reads indexed with it stay in
// the loop instead of being hoisted into registers (which would cost occupancy).
__device__ __forceinline__ int opaque_zero() {
    int z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    return z;
}

// Owned columns [0, nown) of the row come first in its storage: column j's rows are
// at S + j k_t, its coefficient row of X at src[j].
template <typename TB, typename TV, int RL>
__device__ __forceinline__ void coupling_sym_row(int kt, int nown, const TB* __restrict__ S,
                                                 const int* __restrict__ src, const TV* __restrict__ Xh,
                                                 TV* __restrict__ yt, const TV* __restrict__ xt_src,
                                                 TV* __restrict__ part, TV (*red)[3]) {
    constexpr int CG = 64 / RL;          // columns per wave step
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int rl = lane % RL;
    const int cg = lane / RL;
    // X_t rows (zero beyond k_t) staged in the first 64 rows of red
    for (int e = threadIdx.x; e < 64 * kNcomp; e += 256)
        red[e / kNcomp][e % kNcomp] = e < kt * kNcomp ? xt_src[e] : czero<TV>();
    __syncthreads();
    TV acc[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[q][c] = czero<TV>();
    constexpr int U = 2;                 // wave steps whose loads are issued together
    for (int j0 = w * CG; j0 < nown; j0 += 4 * CG * U) {
        int jj[U];
        bool live[U];
        TB sv[U][4];
        TV xl[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            jj[u] = j0 + 4 * CG * u + cg;
            live[u] = jj[u] < nown;
            const TB* col = S + (int64_t)(live[u] ? jj[u] : 0) * kt;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = rl + RL * q;
                if (live[u] && r < kt) sv[u][q] = ldnt(col + r);
                else { sv[u][q].x = 0; sv[u][q].y = 0; }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int sj = live[u] ? src[jj[u]] : 0;
            if constexpr (RL == 4)       // lane rl < 3 fetches component rl; the quad shares it
                xl[u] = (live[u] && rl < 3) ? Xh[(int64_t)sj * kNcomp + rl] : czero<TV>();
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            TV xs[3];
            if constexpr (RL == 4) {
                xs[0] = quad_bcast<0>(xl[u]);
                xs[1] = quad_bcast<1>(xl[u]);
                xs[2] = quad_bcast<2>(xl[u]);
            } else {
                const int sj = live[u] ? src[jj[u]] : 0;
#pragma unroll
                for (int c = 0; c < 3; ++c) xs[c] = live[u] ? Xh[(int64_t)sj * kNcomp + c] : czero<TV>();
            }
            const int z = opaque_zero();     // each step reads the X_t rows afresh
            TV p0 = czero<TV>(), p1 = czero<TV>(), p2 = czero<TV>();
#pragma unroll
            for (int q = 0; q < 4; ++q) {
#pragma unroll
                for (int c = 0; c < 3; ++c) cfma(acc[q][c], sv[u][q], xs[c]);
                const TV* xr = red[rl + RL * q + z];
                cfma(p0, sv[u][q], xr[0]);
                cfma(p1, sv[u][q], xr[1]);
                cfma(p2, sv[u][q], xr[2]);
            }
            p0 = col_sum<RL>(p0);
            p1 = col_sum<RL>(p1);
            p2 = col_sum<RL>(p2);
            // lane rl = c stores component c of the column's partial (selects, no indexing)
            TV o = p2;
            o.x = rl == 1 ? p1.x : o.x;
            o.y = rl == 1 ? p1.y : o.y;
            o.x = rl == 0 ? p0.x : o.x;
            o.y = rl == 0 ? p0.y : o.y;
            if (live[u] && rl < 3) part[(int64_t)jj[u] * kNcomp + rl] = o;
        }
    }
    // Y_t rows: sum over the column groups of each 16-lane row, the 4 rows of the wave
    // and the 4 waves
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            TV v = acc[q][c];
            if constexpr (RL == 4) { v = dpp_add<kDppRor4>(v); v = dpp_add<kDppRor8>(v); }
            if constexpr (RL == 8) v = dpp_add<kDppRor8>(v);
            v.x += shfl_xor_r(v.x, 16);
            v.y += shfl_xor_r(v.y, 16);
            v.x += shfl_xor_r(v.x, 32);
            v.y += shfl_xor_r(v.y, 32);
            acc[q][c] = v;
        }
    __syncthreads();                     // every wave is done with the X_t rows in red
    if (lane < RL)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = rl + RL * q;
            if (r < kt)
#pragma unroll
                for (int c = 0; c < 3; ++c) red[w * 64 + r][c] = acc[q][c];
        }
    __syncthreads();
    for (int e = threadIdx.x; e < kt * kNcomp; e += 256) {
        const int r = e / kNcomp, c = e % kNcomp;
        TV v = cadd(cadd(red[r][c], red[64 + r][c]), cadd(red[128 + r][c], red[192 + r][c]));
        yt[e] = v;
    }
}

// FP64 rows of rank up to 16: the transposed products on the matrix cores, the
// forward product on the vector units, from the same loads.  A 16-column group of the
// owned columns is one 16 x 16 tile: lane l holds column 16 g + l % 16, rows
// 4 s + l / 16 (s < 4) of the block.  Those four values are the A operands of the
// four 16 x 16 x 4 steps of S^T X_t (A[m][k]: column m, row k of the step; B: rows of
// X_t x component, 3 of 16 used; complex in the 3M form), and they also take the lane's
// forward terms S[i][j] X_s[j] for its four rows, summed over the lane's columns and,
// once per row cluster, over the 16 lanes of each DPP row.  Each wave takes every fourth
// group; two groups' loads are in flight.
__device__ __forceinline__ void coupling_sym_mfma16(int kt, int nown, const double2* __restrict__ S,
                                                    const int* __restrict__ src, const double2* __restrict__ Xh,
                                                    double2* __restrict__ yt, const double2* __restrict__ xt_src,
                                                    double2* __restrict__ part, const double2* __restrict__ zero,
                                                    double2 (*red)[3]) {
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int rl = lane & 15, kq = lane >> 4;
    const int ng = (nown + 15) >> 4;
    // B operands of the transposed steps: X_t row 4 s + l / 16, component l % 16
    double2 bt[4];
    double bs[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = 4 * q + kq;
        bt[q] = *(i < kt && rl < kNcomp ? xt_src + i * kNcomp + rl : zero);
        bs[q] = bt[q].x + bt[q].y;
    }
    double2 fa[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) fa[q][c] = czero<double2>();
    struct Grp {
        double2 s[4];
        double2 x[3];
    };
    // the lane's gather index in group g (0 past the end), requested two groups before
    // the group's loads: a load whose address waits for it waits for every older request
    auto gidx = [&](int g) {
        const int j = 16 * g + rl;
        return src[j < nown ? j : 0];
    };
    auto load = [&](int g, int sj) {
        const int j = 16 * g + rl;
        const bool ok = j < nown;
        Grp o;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = 4 * q + kq;
            o.s[q] = *(ok && i < kt ? S + (int64_t)j * kt + i : zero);
        }
        const double2* xs = ok ? Xh + (int64_t)sj * kNcomp : zero;
#pragma unroll
        for (int c = 0; c < 3; ++c) o.x[c] = xs[c];
        return o;
    };
    auto work = [&](const Grp& o, int g) {
        // forward terms of the lane's four rows
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) cfma(fa[q][c], o.s[q], o.x[c]);
        // transposed: D[column][component] over the 16 rows, 3M form
        v4d p1 = {0, 0, 0, 0}, p2 = p1, p3 = p1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            p1 = mfma64(o.s[q].x, bt[q].x, p1);
            p2 = mfma64(o.s[q].y, bt[q].y, p2);
            p3 = mfma64(o.s[q].x + o.s[q].y, bs[q], p3);
        }
        // register r of lane l: column 16 g + 4 r + l / 16, component l % 16
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = 16 * g + 4 * r + kq;
            if (j < nown && rl < kNcomp)
                part[(int64_t)j * kNcomp + rl] = make_double2(p1[r] - p2[r], p3[r] - p1[r] - p2[r]);
        }
    };
    const int mine = ng > w ? (ng - 1 - w) / 4 + 1 : 0;
    if (mine > 0) {
        int ga = gidx(w), gb = gidx(w + 4);
        Grp a = load(w, ga), b = load(w + 4, gb);
        ga = gidx(w + 8);
        gb = gidx(w + 12);
        for (int i = 0; i < mine; i += 2) {
            const int g = w + 4 * i;
            work(a, g);
            a = load(g + 8, ga);
            ga = gidx(g + 16);
            __builtin_amdgcn_sched_barrier(0);
            work(b, g + 4);              // past this wave's last group: zeros, nothing stored
            b = load(g + 12, gb);
            gb = gidx(g + 20);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // forward rows: sum over the 16 lanes of each DPP row, then over the 4 waves
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) fa[q][c] = col_sum<16>(fa[q][c]);
    if (rl == 0)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) red[w * 16 + 4 * q + kq][c] = fa[q][c];
    __syncthreads();
    for (int e = threadIdx.x; e < kt * kNcomp; e += 256) {
        const int r = e / kNcomp, c = e % kNcomp;
        yt[e] = cadd(cadd(red[r][c], red[16 + r][c]), cadd(red[32 + r][c], red[48 + r][c]));
    }
}

template <typename TB, typename TV>
__global__ __launch_bounds__(256) void k_coupling_sym(const int* __restrict__ row_cl, const int64_t* __restrict__ row_off,
                                                      const int* __restrict__ row_colptr, const int* __restrict__ colsrc,
                                                      const int* __restrict__ row_nown, const int* __restrict__ row_pbase,
                                                      const int* __restrict__ cl_rank, const int* __restrict__ cl_coef,
                                                      const TB* __restrict__ coupling, const TV* __restrict__ Xh,
                                                      TV* __restrict__ Yh, TV* __restrict__ part,
                                                      const double2* __restrict__ zero) {
    __shared__ TV red[256][3];
    const int slot = blockIdx.x;
    const int t = row_cl[slot];
    const int kt = cl_rank[t];
    const int nown = row_nown[slot];
    const TB* S = coupling + row_off[slot];
    const int co = cl_coef[t];
    const int* src = colsrc + row_colptr[slot];
    TV* pt = part + (int64_t)row_pbase[slot] * kNcomp;
    const TV* xt = Xh + (int64_t)co * kNcomp;
    TV* yt = Yh + (int64_t)co * kNcomp;
    if constexpr (std::is_same<TV, double2>::value && std::is_same<TB, double2>::value) {
        if (kt <= 16) {
            coupling_sym_mfma16(kt, nown, S, src, Xh, yt, xt, pt, zero, red);
            return;
        }
    }
    if (kt <= 16)
        coupling_sym_row<TB, TV, 4>(kt, nown, S, src, Xh, yt, xt, pt, red);
    else if (kt <= 32)
        coupling_sym_row<TB, TV, 8>(kt, nown, S, src, Xh, yt, xt, pt, red);
    else
        coupling_sym_row<TB, TV, 16>(kt, nown, S, src, Xh, yt, xt, pt, red);
}

// Y_s += the partials S_ts^T X_t of the blocks that land in row slot s (fixed order).
template <typename TV>
__global__ __launch_bounds__(64) void k_coupling_recv(const int* __restrict__ row_cl, const int* __restrict__ rptr,
                                                      const int* __restrict__ rp, const int* __restrict__ cl_rank,
                                                      const int* __restrict__ cl_coef, const TV* __restrict__ part,
                                                      TV* __restrict__ Yh) {
    const int slot = blockIdx.x;
    const int a = rptr[slot], b = rptr[slot + 1];
    if (a == b) return;
    const int t = row_cl[slot];
    const int n3 = cl_rank[t] * kNcomp;
    TV* y = Yh + (int64_t)cl_coef[t] * kNcomp;
    for (int e = threadIdx.x; e < n3; e += 64) {
        TV acc = czero<TV>();
#pragma unroll 8
        for (int q = a; q < b; ++q) acc = cadd(acc, part[(int64_t)rp[q] * kNcomp + e]);
        y[e] = cadd(y[e], acc);
    }
}

// ---------------------------------------------------------------- downward pass
// Y_c[b][c] += sum_a T_c[b, a] Y_p[a][c]
template <typename TB, typename TV>
__global__ __launch_bounds__(64) void k_transfer_down(const int* __restrict__ list, const int* __restrict__ cl_rank,
                                                      const int* __restrict__ cl_coef, const int* __restrict__ cl_parent,
                                                      const int64_t* __restrict__ cl_toff, const TB* __restrict__ transfer,
                                                      TV* __restrict__ Yh) {
    const int ch = list[blockIdx.x];
    const int p = cl_parent[ch];
    const int kc = cl_rank[ch], kp = cl_rank[p];
    const TB* T = transfer + cl_toff[ch];
    const TV* yp = Yh + (int64_t)cl_coef[p] * kNcomp;
    for (int b = threadIdx.x; b < kc; b += 64) {
        TV acc0 = czero<TV>(), acc1 = czero<TV>(), acc2 = czero<TV>();
#pragma unroll 8
        for (int a = 0; a < kp; ++a) {
            TB tv = T[(int64_t)a * kc + b];
            cfma(acc0, tv, yp[a * 3 + 0]);
            cfma(acc1, tv, yp[a * 3 + 1]);
            cfma(acc2, tv, yp[a * 3 + 2]);
        }
        TV* o = Yh + (int64_t)(cl_coef[ch] + b) * kNcomp;
        o[0] = cadd(o[0], acc0); o[1] = cadd(o[1], acc1); o[2] = cadd(o[2], acc2);
    }
}

// Row `lane` of leaf t after a near pass (s0..s2: this pass's sums): with several
// passes, the earlier ones leave their sums in ypart and stop; the last adds them,
// the backward transformation V_t Y_t and the epilogue z = x + alpha y (op Z).
template <typename TB, typename TV>
__device__ __forceinline__ void near_finish_row(int t, int n, int lane, TV s0, TV s1, TV s2, int pass, int npass,
                                                TV* __restrict__ ypart, const int* __restrict__ cl_rank,
                                                const int* __restrict__ cl_coef, const int* __restrict__ cl_begin,
                                                const int64_t* __restrict__ cl_basis_off, const TB* __restrict__ basis,
                                                const TV* __restrict__ Yh, const int* __restrict__ perm,
                                                const TV* __restrict__ x, TV* __restrict__ y, int op,
                                                typename Real<TV>::T alpha) {
    if (npass > 1) {   // rows of the earlier passes; all but the last pass stop here
        TV* yp = ypart + (int64_t)(cl_begin[t] + lane) * kNcomp;
        if (pass > 0) {
            s0 = cadd(yp[0], s0);
            s1 = cadd(yp[1], s1);
            s2 = cadd(yp[2], s2);
        }
        if (pass < npass - 1) {
            yp[0] = s0;
            yp[1] = s1;
            yp[2] = s2;
            return;
        }
    }
    const int k = cl_rank[t];
    if (k > 0) {   // backward transformation at the leaf: y_t += V_t Y_t
        const TB* V = basis + cl_basis_off[t];
        const TV* yt = Yh + (int64_t)cl_coef[t] * kNcomp;
        for (int a = 0; a < k; ++a) {
            TB v = V[(int64_t)a * n + lane];
            cfma(s0, v, yt[a * 3 + 0]);
            cfma(s1, v, yt[a * 3 + 1]);
            cfma(s2, v, yt[a * 3 + 2]);
        }
    }
    const int vox = perm[cl_begin[t] + lane];
    TV* yo = y + (int64_t)vox * kNcomp;
    if (op == 1) {
        const TV* xi = x + (int64_t)vox * kNcomp;
        TV r;
        r.x = xi[0].x + alpha * s0.x; r.y = xi[0].y + alpha * s0.y; yo[0] = r;
        r.x = xi[1].x + alpha * s1.x; r.y = xi[1].y + alpha * s1.y; yo[1] = r;
        r.x = xi[2].x + alpha * s2.x; r.y = xi[2].y + alpha * s2.y; yo[2] = r;
    } else {
        yo[0] = s0; yo[1] = s1; yo[2] = s2;
    }
}

// ---------------------------------------------------------------- near field + leaf backward + epilogue
// One 256-thread group per leaf t; wave w streams near blocks w, w+4, ...;
// lane i owns row i of every block (column-major blocks: coalesced columns).
// With several passes (pass_ptr set), this launch covers pass `pass` of the
// leaf's blocks: the earlier passes leave their row sums in ypart (tree order),
// the last one adds them and finishes.
template <typename TB, typename TV, bool NT>
__global__ __launch_bounds__(256) void k_near_epilogue(
    const int* __restrict__ pass_ptr, int pass, int npass, TV* __restrict__ ypart,
    const int* __restrict__ leaf_id, const int* __restrict__ near_ptr, const int* __restrict__ near_sbeg,
    const int* __restrict__ near_ssize, const int64_t* __restrict__ near_off, const TB* __restrict__ near,
    const int* __restrict__ cl_rank, const int* __restrict__ cl_coef, const int* __restrict__ cl_begin,
    const int* __restrict__ cl_size, const int64_t* __restrict__ cl_basis_off, const TB* __restrict__ basis,
    const TV* __restrict__ U, const TV* __restrict__ Yh, const int* __restrict__ perm, const TV* __restrict__ x,
    TV* __restrict__ y, int op, typename Real<TV>::T alpha) {
    __shared__ TV red[4][kMaxLeaf][3];
    const int slot = blockIdx.x;
    const int t = leaf_id[slot];
    const int n = cl_size[t];
    const int lane = threadIdx.x & 63;
    // wave index as a wave-uniform value: block metadata and source values then
    // come through scalar loads, and only the block stream uses vector loads
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    TV acc0 = czero<TV>(), acc1 = czero<TV>(), acc2 = czero<TV>();
    const int b0 = pass_ptr ? pass_ptr[slot * (npass + 1) + pass] : near_ptr[slot];
    const int e = pass_ptr ? pass_ptr[slot * (npass + 1) + pass + 1] : near_ptr[slot + 1];
    for (int blk = b0 + w; blk < e; blk += 4) {
        const int sb = near_sbeg[blk];
        const int ns = near_ssize[blk];
        const TB* Gb = near + near_off[blk] + lane;
        const TV* us = U + (int64_t)sb * kNcomp;
        if (lane < n) {
#pragma unroll 16
            for (int j = 0; j < ns; ++j) {
                TB gv = ldblk<NT>(Gb + (int64_t)j * n);
                cfma(acc0, gv, us[j * 3 + 0]);
                cfma(acc1, gv, us[j * 3 + 1]);
                cfma(acc2, gv, us[j * 3 + 2]);
            }
        }
    }
    red[w][lane][0] = acc0; red[w][lane][1] = acc1; red[w][lane][2] = acc2;
    __syncthreads();
    if (w == 0 && lane < n) {
        TV s0 = cadd(cadd(red[0][lane][0], red[1][lane][0]), cadd(red[2][lane][0], red[3][lane][0]));
        TV s1 = cadd(cadd(red[0][lane][1], red[1][lane][1]), cadd(red[2][lane][1], red[3][lane][1]));
        TV s2 = cadd(cadd(red[0][lane][2], red[1][lane][2]), cadd(red[2][lane][2], red[3][lane][2]));
        near_finish_row<TB, TV>(t, n, lane, s0, s1, s2, pass, npass, ypart, cl_rank, cl_coef, cl_begin,
                                cl_basis_off, basis, Yh, perm, x, y, op, alpha);
    }
}

// ---------------------------------------------------------------- tiled near field on the matrix cores
// Full-mode near field over stored-once blocks: a tile is kTileLeaves target leaves
// consecutive in tree order, walked as a list of steps; a step is one stored block G
// (n_t x n_s, column-major) and, for each target slot j, the source leaf whose U_s it
// multiplies (or none).  G is read once per step for all the tile's targets instead of
// once per leaf pair.  Products on the matrix cores (A = 16 rows x 4 columns of G, B = 4
// rows of U_s x 16 target slots, one 16 x 16 tile per field component); the complex
// product takes four real ones (re += Gr Ur - Gi Ui, im += Gr Ui + Gi Ur) or, in the 3M
// form, three (see tile_mma).  k_near_tile_split runs the steps (a form for full 64 x 64
// blocks and one for any shape); k_near_tile_finish finishes every target's rows as
// k_near_epilogue does.
// complex products as three real ones (the 3M form: Gr Ur, Gi Ui, (Gr + Gi)(Ur + Ui))
// instead of four
constexpr bool kTile3M = true;

// Precision of the tiled products: FP64 (v_mfma_f64_16x16x4f64) or FP32
// (v_mfma_f32_16x16x4f32), same operand layouts (lane l: A[l % 16][l / 16],
// B[l / 16][l % 16]); result register r of lane l is row drow(r, l / 16), column
// l % 16, with drow = 4 r + l / 16 in FP64 and 4 (l / 16) + r in FP32 (both checked on
// the device).
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename TV> struct Tile;
template <> struct Tile<double2> {
    using R = double;
    using V4 = v4d;
    __device__ static V4 mma(double a, double b, V4 c) { return mfma64(a, b, c); }
    __device__ static int drow(int r, int kq) { return 4 * r + kq; }
};
template <> struct Tile<float2> {
    using R = float;
    using V4 = v4f;
    __device__ static V4 mma(float a, float b, V4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int drow(int r, int kq) { return 4 * kq + r; }
};

template <typename TV> __device__ __forceinline__ TV cmake(typename Real<TV>::T x, typename Real<TV>::T y) {
    TV v;
    v.x = x;
    v.y = y;
    return v;
}

// One k step's operands: 4 columns of G (16 rows a wave) and the matching 4 rows of
// the 16 sources, for the three field components.
template <typename TV> struct TileOps {
    TV a, u0, u1, u2;
};

// acc[c][q], component c: with four real products q = 0 re, 1 im; with three (M3,
// the 3M form) q = 0 Gr Ur, 1 Gi Ui, 2 (Gr + Gi)(Ur + Ui), so re = [0] - [1] and
// im = [2] - [0] - [1]
template <bool M3, typename TV>
__device__ __forceinline__ void tile_mma(const TileOps<TV>& o, typename Tile<TV>::V4 (&acc)[3][3]) {
    using T = Tile<TV>;
    const TV u[3] = {o.u0, o.u1, o.u2};
    if constexpr (M3) {
        const auto sa = o.a.x + o.a.y;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            acc[c][0] = T::mma(o.a.x, u[c].x, acc[c][0]);
            acc[c][1] = T::mma(o.a.y, u[c].y, acc[c][1]);
            acc[c][2] = T::mma(sa, u[c].x + u[c].y, acc[c][2]);
        }
    } else {
        const auto nai = -o.a.y;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            acc[c][0] = T::mma(o.a.x, u[c].x, acc[c][0]);
            acc[c][1] = T::mma(o.a.x, u[c].y, acc[c][1]);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            acc[c][0] = T::mma(nai, u[c].y, acc[c][0]);
            acc[c][1] = T::mma(o.a.y, u[c].x, acc[c][1]);
        }
    }
}

// FP32 sums each step's products (one stored block times its sources) in accumulators
// of their own and adds them to running totals at the step's end: a block product,
// then a sum over blocks, as the tier's error bound assumes.  FP64 chains every step
// in the same accumulators (tot is unused).
template <bool M3, typename TV>
__device__ __forceinline__ void tile_flush(typename Tile<TV>::V4 (&acc)[3][3], typename Tile<TV>::V4 (&tot)[3][3]) {
    if constexpr (!std::is_same<TV, double2>::value) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q = 0; q < (M3 ? 3 : 2); ++q) {
                tot[c][q] += acc[c][q];
                acc[c][q] = typename Tile<TV>::V4{0, 0, 0, 0};
            }
    }
}
// the sums of all steps back in acc
template <bool M3, typename TV>
__device__ __forceinline__ void tile_total(typename Tile<TV>::V4 (&acc)[3][3], typename Tile<TV>::V4 (&tot)[3][3]) {
    if constexpr (!std::is_same<TV, double2>::value) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q = 0; q < (M3 ? 3 : 2); ++q) acc[c][q] = tot[c][q];
    }
}

// Two groups of four waves per tile, taking alternate
// steps, so that a CU holds two groups whose step boundaries (two barriers each: the
// buffer's reads done, then its refill) fall at different times and one keeps the
// matrix cores busy while the other refills.  Wave w owns rows 16 w .. + 15 and all 64
// columns of the block; the group's sources are staged in one LDS buffer; the A
// operand runs two k steps ahead across steps.  Group h leaves its sums in part[h]
// (tree order); k_near_tile_finish adds the two and finishes the rows.
// FULL = false takes blocks of any shape n_t x n_s (leaves under 64 voxels): source rows
// past n_s are staged as zeros, A reads clamp the column to n_s - 1 (a finite value
// times a zero row) and the row to 0 past n_t (rows that are never stored), and a wave
// skips the products of k steps past n_s and of rows it holds past n_t.
template <typename TV, bool M3, bool FULL>
__global__ __launch_bounds__(256, 2) void k_near_tile_split(
    const int* __restrict__ tile_ptr, const int* __restrict__ tile_leaf, const int64_t* __restrict__ step_off,
    const int* __restrict__ step_shape, const int* __restrict__ step_src, const TV* __restrict__ near,
    const TV* __restrict__ zsrc,
    const int* __restrict__ cl_begin, const int* __restrict__ cl_size, const TV* __restrict__ U,
    TV* __restrict__ part0, TV* __restrict__ part1) {
    constexpr int kSlice = kMaxLeaf * kNcomp;
    constexpr int kChunks = kTileLeaves * kSlice / 256;        // entries each thread stages per step
    constexpr int kSteps = kMaxLeaf / 4;                       // k steps of 4 columns
    constexpr int kRowStride = kTileLeaves * kNcomp;
    __shared__ TV stage[kMaxLeaf][kTileLeaves][kNcomp];
    const int tile = blockIdx.x >> 1, h = blockIdx.x & 1;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rl = lane & 15, kq = lane >> 4;
    const int row = 16 * w + rl;
    typename Tile<TV>::V4 acc[3][3], tot[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[c][q] = tot[c][q] = typename Tile<TV>::V4{0, 0, 0, 0};
    const int b = tile_ptr[tile] + h, e = tile_ptr[tile + 1];
    if (b < e) {
        int sb[kChunks];
        int ns_f = kMaxLeaf;                                    // columns of the block whose sources sb holds
        TV sv[kChunks];
        auto srcs = [&](int st) {
#pragma unroll
            for (int j = 0; j < kChunks; ++j) sb[j] = step_src[(int64_t)st * kTileLeaves + (tid + 256 * j) / kSlice];
            if constexpr (!FULL) ns_f = step_shape[st] >> 16;
        };
        auto fetch = [&]() {
#pragma unroll
            for (int j = 0; j < kChunks; ++j) {
                const int o = (tid + 256 * j) % kSlice;
                sv[j] = *(sb[j] >= 0 && (FULL || o / kNcomp < ns_f) ? U + (int64_t)sb[j] * kNcomp + o : zsrc);
            }
        };
        auto store = [&]() {
#pragma unroll
            for (int j = 0; j < kChunks; ++j) {
                const int i = tid + 256 * j;
                const int n = i / kSlice, o = i % kSlice;
                TV v = sv[j];
                asm volatile("" : "+v"(v.x), "+v"(v.y));
                stage[o / kNcomp][n][o % kNcomp] = v;
            }
        };
        const int mine = b + ((e - 1 - b) >> 1) * 2;              // this group's last step
        auto last = [&](int st) { return st < e ? st : mine; };   // past the end: re-read the last
        auto aptr = [&](int st) { return near + step_off[st] + row + (int64_t)kq * kMaxLeaf; };
        // general shapes: the step's block at row min(row, 0 past n_t), its rows n_t apart,
        // column 4 m + kq of k step m clamped to n_s - 1
        struct Blk {
            const TV* p;
            int nt, ns;
        };
        auto blk = [&](int st) {
            const int sh = step_shape[st];
            Blk o;
            o.nt = sh & 0xffff;
            o.ns = sh >> 16;
            o.p = near + step_off[st] + (row < o.nt ? row : 0);
            return o;
        };
        auto aload = [&](const Blk& o, int m) { return o.p[(int64_t)min(4 * m + kq, o.ns - 1) * o.nt]; };
        srcs(b);
        fetch();
        store();
        srcs(last(b + 2));
        const TV* ga = aptr(b);
        Blk ca, na;
        TV a0, a1;
        if constexpr (FULL) {
            a0 = ga[0];
            a1 = ga[4 * kMaxLeaf];
        } else {
            ca = blk(b);
            a0 = aload(ca, 0);
            a1 = aload(ca, 1);
        }
        __syncthreads();
        for (int st = b; st < e; st += 2) {
            fetch();                                            // slices of step st + 2
            srcs(last(st + 4));
            const TV* gn = aptr(last(st + 2));
            if constexpr (!FULL) na = blk(last(st + 2));
            const TV* bs = &stage[0][0][0] + (kq * kTileLeaves + rl) * kNcomp;
            TV bu[2][3];
#pragma unroll
            for (int c = 0; c < 3; ++c) bu[0][c] = bs[c];
#pragma unroll
            for (int i = 0; i < kSteps; ++i) {
                if (i + 1 < kSteps) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) bu[(i + 1) & 1][c] = bs[(i + 1) * 4 * kRowStride + c];
                }
                TileOps<TV> o;
                o.a = (i & 1) ? a1 : a0;
                o.u0 = bu[i & 1][0];
                o.u1 = bu[i & 1][1];
                o.u2 = bu[i & 1][2];
                if (FULL || (4 * i < ca.ns && 16 * w < ca.nt)) tile_mma<M3, TV>(o, acc);
                TV an;
                if constexpr (FULL) {
                    an = *(i + 2 < kSteps ? ga + (i + 2) * 4 * kMaxLeaf : gn + (i + 2 - kSteps) * 4 * kMaxLeaf);
                } else {
                    an = i + 2 < kSteps ? aload(ca, i + 2) : aload(na, i + 2 - kSteps);
                }
                if (i & 1)
                    a1 = an;
                else
                    a0 = an;
                __builtin_amdgcn_sched_barrier(0);
            }
            tile_flush<M3, TV>(acc, tot);
            ga = gn;
            if constexpr (!FULL) ca = na;
            __syncthreads();                                    // every wave is done with the buffer
            store();
            __syncthreads();
        }
        tile_total<M3, TV>(acc, tot);
    }
    // sums to this group's partial buffer: register r of lane l is row drow(r, l / 16) of
    // the wave's 16, slot l % 16
    TV* out = h ? part1 : part0;
    const int t = tile_leaf[tile * kTileLeaves + rl];
    if (t >= 0) {
        const int n = cl_size[t];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * w + Tile<TV>::drow(r, kq);
            if (i < n) {
                TV* o = out + (int64_t)(cl_begin[t] + i) * kNcomp;
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    o[c] = M3 ? cmake<TV>(acc[c][0][r] - acc[c][1][r], acc[c][2][r] - acc[c][0][r] - acc[c][1][r])
                              : cmake<TV>(acc[c][0][r], acc[c][1][r]);
            }
        }
    }
}

// The rows of leaf slot blockIdx.x: the two split groups' sums, the leaf backward
// transformation and the epilogue (as k_near_epilogue's last pass).
template <typename TV>
__global__ __launch_bounds__(64) void k_near_tile_finish(
    const int* __restrict__ leaf_id, const TV* __restrict__ part0, const TV* __restrict__ part1,
    const int* __restrict__ cl_rank, const int* __restrict__ cl_coef, const int* __restrict__ cl_begin,
    const int* __restrict__ cl_size, const int64_t* __restrict__ cl_basis_off, const TV* __restrict__ basis,
    const TV* __restrict__ Yh, const int* __restrict__ perm, const TV* __restrict__ x,
    TV* __restrict__ y, int op, typename Real<TV>::T alpha) {
    const int t = leaf_id[blockIdx.x];
    const int n = cl_size[t];
    const int lane = threadIdx.x;
    if (lane >= n) return;
    const int64_t i = (int64_t)(cl_begin[t] + lane) * kNcomp;
    near_finish_row<TV, TV>(t, n, lane, cadd(part0[i], part1[i]), cadd(part0[i + 1], part1[i + 1]),
                                      cadd(part0[i + 2], part1[i + 2]), 0, 1, nullptr, cl_rank, cl_coef, cl_begin,
                                      cl_basis_off, basis, Yh, perm, x, y, op, alpha);
}

// ---------------------------------------------------------------- symmetric near field
// Sum over the 16 lanes of each DPP row (rotations by 8, 4, 2, 1): every lane of
// the row ends with the row's sum.  All 64 lanes must be active.
template <int R> __device__ __forceinline__ double ror_row(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, 0x120 + R, 0xf, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, 0x120 + R, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
template <int R> __device__ __forceinline__ float ror_row(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x120 + R, 0xf, 0xf, false));
}
template <typename T> __device__ __forceinline__ T rowsum16(T v) {
    v += ror_row<8>(v);
    v += ror_row<4>(v);
    v += ror_row<2>(v);
    v += ror_row<1>(v);
    return v;
}

// One group per leaf t (launch slot); its four waves take t's owned blocks in
// turn (the diagonal block, then the pairs t streams for both leaves).  Lane
// (cg = lane / 16, rg = lane % 16) holds rows rg + 16 q (q < 4) of t and, in
// panel k of four columns, column j = 4 k + cg of the block:
//   own rows      acc[q] += G(rg + 16 q, j) u_s(j)           (summed over cg at the end)
//   other leaf    part(j) = sum_i G(i, j) u_t(i)             (DPP row sum over rg)
// Own rows go to rows (tree order), the other leaf's to its partial slot.
template <typename TB, typename TV, bool NT>
__global__ __launch_bounds__(256) void k_near_sym(const int* __restrict__ sym_leaf, const int* __restrict__ sym_ptr,
                                                  const int* __restrict__ sym_sbeg, const int* __restrict__ sym_ssize,
                                                  const int64_t* __restrict__ sym_off, const int* __restrict__ sym_pslot,
                                                  const TB* __restrict__ near, const int* __restrict__ cl_begin,
                                                  const int* __restrict__ cl_size, const TV* __restrict__ U,
                                                  TV* __restrict__ rows, TV* __restrict__ part) {
    __shared__ TV red[4][kMaxLeaf][3];
    __shared__ TV ut[kMaxLeaf][3];               // u_t, read by every column product
    const int slot = blockIdx.x;
    const int t = sym_leaf[slot];
    const int n = cl_size[t], tb = cl_begin[t];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int rg = lane & 15, cg = lane >> 4;
    if (threadIdx.x < kMaxLeaf * 3)
        ut[threadIdx.x / 3][threadIdx.x % 3] =
            threadIdx.x < n * 3 ? U[(int64_t)tb * kNcomp + threadIdx.x] : czero<TV>();
    TV acc[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[q][c] = czero<TV>();
    __syncthreads();
    const int e = sym_ptr[slot + 1];
    for (int blk = sym_ptr[slot] + w; blk < e; blk += 4) {
        const int sb = sym_sbeg[blk];
        const int ns = sym_ssize[blk];
        const int ps = sym_pslot[blk];
        const TB* G = near + sym_off[blk];
        const TV* us = U + (int64_t)sb * kNcomp;
        // panel k holds columns 4k .. 4k + 3.  Loads have no branches or selects:
        // entries outside the block read the block's first entry (finite), which
        // meets a zero (u_t beyond n in LDS, u_s beyond ns masked where it is used)
        // or lands in a row or column that is not stored.  Column 4k + cg of the
        // other leaf is kept by lane rg = k and stored once per block.
        TV keep[3];
        auto load_panel = [&](int k, TB* dst, TV* du) {
            const int j = 4 * k + cg;
            const bool jv = j < ns;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = rg + 16 * q;
                dst[q] = ldblk<NT>(G + ((jv && i < n) ? (int64_t)j * n + i : 0));
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) du[c] = us[jv ? j * 3 + c : c];
        };
        auto panel = [&](int k, const TB* g, const TV* u) {
            const bool jv = 4 * k + cg < ns;
            TV um[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                um[c].x = jv ? u[c].x : 0;
                um[c].y = jv ? u[c].y : 0;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c) cfma(acc[q][c], g[q], um[c]);
            if (ps >= 0) {   // wave-uniform: off-diagonal pair, the other leaf's rows
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    TV p = czero<TV>();
#pragma unroll
                    for (int q = 0; q < 4; ++q) cfma(p, g[q], ut[rg + 16 * q][c]);
                    p.x = rowsum16(p.x);
                    p.y = rowsum16(p.y);
                    keep[c].x = rg == k ? p.x : keep[c].x;
                    keep[c].y = rg == k ? p.y : keep[c].y;
                }
            }
        };
#pragma unroll
        for (int c = 0; c < 3; ++c) keep[c] = czero<TV>();
        // one panel at a time: latency is hidden by the other waves of the SIMD
        const int npan = (ns + 3) >> 2;
        for (int k = 0; k < npan; ++k) {
            TB g[4];
            TV u[3];
            load_panel(k, g, u);
            panel(k, g, u);
        }
        const int jk = 4 * rg + cg;
        if (ps >= 0 && jk < ns) {
            TV* pj = part + ((int64_t)ps * kMaxLeaf + jk) * kNcomp;
            pj[0] = keep[0];
            pj[1] = keep[1];
            pj[2] = keep[2];
        }
    }
    // own rows: sum over the four column groups of the wave, then over the waves
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            acc[q][c].x += __shfl_xor(acc[q][c].x, 16);
            acc[q][c].y += __shfl_xor(acc[q][c].y, 16);
            acc[q][c].x += __shfl_xor(acc[q][c].x, 32);
            acc[q][c].y += __shfl_xor(acc[q][c].y, 32);
        }
    if (cg == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = rg + 16 * q;
            if (i < n)
#pragma unroll
                for (int c = 0; c < 3; ++c) red[w][i][c] = acc[q][c];
        }
    }
    __syncthreads();
    if (threadIdx.x < n) {
        const int i = threadIdx.x;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            TV s = cadd(cadd(red[0][i][c], red[1][i][c]), cadd(red[2][i][c], red[3][i][c]));
            rows[(int64_t)(tb + i) * kNcomp + c] = s;
        }
    }
}

// One wave per leaf: own rows + the partials other leaves wrote for it (fixed
// order) + V_t Y_t, then the epilogue, as k_near_epilogue.
template <typename TB, typename TV>
__global__ __launch_bounds__(64) void k_near_sym_finish(
    const int* __restrict__ sym_leaf, const int* __restrict__ in_ptr, const int* __restrict__ in_slot,
    const TV* __restrict__ rows, const TV* __restrict__ part, const int* __restrict__ cl_rank,
    const int* __restrict__ cl_coef, const int* __restrict__ cl_begin, const int* __restrict__ cl_size,
    const int64_t* __restrict__ cl_basis_off, const TB* __restrict__ basis, const TV* __restrict__ Yh,
    const int* __restrict__ perm, const TV* __restrict__ x, TV* __restrict__ y, int op, typename Real<TV>::T alpha) {
    const int slot = blockIdx.x;
    const int t = sym_leaf[slot];
    const int n = cl_size[t];
    const int lane = threadIdx.x;
    if (lane >= n) return;
    const int64_t r = (int64_t)(cl_begin[t] + lane) * kNcomp;
    TV s0 = rows[r], s1 = rows[r + 1], s2 = rows[r + 2];
    const int e = in_ptr[slot + 1];
#pragma unroll 4
    for (int k = in_ptr[slot]; k < e; ++k) {
        const TV* p = part + ((int64_t)in_slot[k] * kMaxLeaf + lane) * kNcomp;
        s0 = cadd(s0, p[0]);
        s1 = cadd(s1, p[1]);
        s2 = cadd(s2, p[2]);
    }
    const int k = cl_rank[t];
    if (k > 0) {   // backward transformation at the leaf: y_t += V_t Y_t
        const TB* V = basis + cl_basis_off[t];
        const TV* yt = Yh + (int64_t)cl_coef[t] * kNcomp;
        for (int a = 0; a < k; ++a) {
            TB v = V[(int64_t)a * n + lane];
            cfma(s0, v, yt[a * 3 + 0]);
            cfma(s1, v, yt[a * 3 + 1]);
            cfma(s2, v, yt[a * 3 + 2]);
        }
    }
    const int vox = perm[cl_begin[t] + lane];
    TV* yo = y + (int64_t)vox * kNcomp;
    if (op == 1) {
        const TV* xi = x + (int64_t)vox * kNcomp;
        TV o;
        o.x = xi[0].x + alpha * s0.x; o.y = xi[0].y + alpha * s0.y; yo[0] = o;
        o.x = xi[1].x + alpha * s1.x; o.y = xi[1].y + alpha * s1.y; yo[1] = o;
        o.x = xi[2].x + alpha * s2.x; o.y = xi[2].y + alpha * s2.y; yo[2] = o;
    } else {
        yo[0] = s0; yo[1] = s1; yo[2] = s2;
    }
}

// ---------------------------------------------------------------- launcher
template <typename TB, typename TV>
static hipError_t matvec_tier(const DevH2& d, const LevelLaunch& lv, int op, const TierData& td, const TV* x,
                              TV* y, int64_t n_rhs, int64_t ld, hipStream_t s, Profiler* prof) {
    using R = typename Real<TV>::T;
    const TB* near = (const TB*)td.near;
    const TB* coupling = (const TB*)td.coupling;
    const TB* basis = (const TB*)td.basis;
    const TB* transfer = (const TB*)td.transfer;
    TV* U = (TV*)d.U;
    TV* Xh = (TV*)d.Xh;
    TV* Yh = (TV*)d.Yh;
    const R alpha = (R)(d.sigma * d.k * d.k * d.volume);
    auto begin = [&](int f) { if (prof) prof->begin(f, s); };
    auto end = [&](int f) { if (prof) prof->end(f, s); };
    // full mode over stored-once blocks: all passes but the last read only U, so they
    // run on the side stream beside the upward pass, couplings and downward pass (when
    // the kernel families are timed, those passes are timed on the side stream)
    constexpr bool same = std::is_same<TV, TB>::value;     // FP64 or FP32 throughout
    const bool tiles = same && d.near_tiles && !d.near_sym;
    const bool overlap = !d.near_sym && d.near_side && (tiles || d.near_passes > 1);
    auto near_tile = [&](int part, const TV* xr, TV* yr, hipStream_t st) {
        if constexpr (same) {
            if (part != 1) {
                auto split = d.tiles_full ? k_near_tile_split<TV, kTile3M, true> : k_near_tile_split<TV, kTile3M, false>;
                split<<<2 * d.n_tiles, 256, 0, st>>>(d.tile_ptr, d.tile_leaf, d.step_off, d.step_shape, d.step_src,
                                                     near, (const TV*)d.zero_block, d.cl_begin, d.cl_size, U,
                                                     (TV*)d.near_ypart, (TV*)d.tile_part1);
            }
            if (part != 0)
                k_near_tile_finish<TV><<<d.n_leaves, 64, 0, st>>>(
                    d.leaf_id, (const TV*)d.near_ypart, (const TV*)d.tile_part1, d.cl_rank, d.cl_coef, d.cl_begin,
                    d.cl_size, d.cl_basis_off, basis, Yh, d.perm, xr, yr, op, alpha);
        }
    };
    auto near_kernel = d.near_cached ? k_near_epilogue<TB, TV, false> : k_near_epilogue<TB, TV, true>;
    auto near_pass = [&](int pass, const TV* xr, TV* yr, hipStream_t st) {
        const int np = d.near_passes;
        near_kernel<<<d.n_leaves, 256, 0, st>>>(np > 1 ? d.near_pass_ptr : nullptr, pass, np, (TV*)d.near_ypart,
                                                d.leaf_id, d.near_ptr, d.near_sbeg, d.near_ssize, d.near_off, near,
                                                d.cl_rank, d.cl_coef, d.cl_begin, d.cl_size, d.cl_basis_off, basis, U,
                                                Yh, d.perm, xr, yr, op, alpha);
    };
    for (int64_t r = 0; r < n_rhs; ++r) {
        const TV* xr = x + r * ld;
        TV* yr = y + r * ld;
        begin(0);
        k_prologue<TV><<<(d.n_vox + 255) / 256, 256, 0, s>>>(d.n_vox, d.perm, d.chi, xr, U, op);
        end(0);
        if (overlap) {
            hipError_t e = hipEventRecord(d.near_fork, s);
            if (e == hipSuccess) e = hipStreamWaitEvent(d.near_side, d.near_fork, 0);
            if (e != hipSuccess) return e;
            if (prof) prof->begin(5, d.near_side);
            if (tiles)
                near_tile(0, xr, yr, d.near_side);
            else
                for (int pass = 0; pass + 1 < d.near_passes; ++pass) near_pass(pass, xr, yr, d.near_side);
            if (prof) prof->end(5, d.near_side);
            if ((e = hipEventRecord(d.near_join, d.near_side)) != hipSuccess) return e;
        }
        if (d.coef_rows > 0) {
            begin(1);
            k_leaf_forward<TB, TV><<<d.n_leaves, 64, 0, s>>>(d.leaf_id, d.cl_rank, d.cl_coef, d.cl_begin, d.cl_size,
                                                             d.cl_basis_off, basis, U, Xh);
            end(1);
            begin(2);
            for (int l = 0; l < lv.n_up; ++l)
                if (lv.up_count[l] > 0)
                    k_transfer_up<TB, TV><<<lv.up_count[l], 64, 0, s>>>(d.up_list + lv.up_begin[l], d.cl_rank, d.cl_coef,
                                                                        d.cl_first_child, d.cl_nchild, d.cl_transfer_off,
                                                                        transfer, Xh);
            end(2);
            begin(3);
            if (d.coup_sym) {
                k_coupling_sym<TB, TV><<<d.n_rowcl, 256, 0, s>>>(d.row_cl, d.row_off, d.row_colptr, d.colsrc,
                                                                 d.row_nown, d.row_pbase, d.cl_rank, d.cl_coef,
                                                                 coupling, Xh, Yh, (TV*)d.cpart,
                                                                 (const double2*)d.zero_block);
                end(3);
                begin(7);
                k_coupling_recv<TV><<<d.n_rowcl, 64, 0, s>>>(d.row_cl, d.crecv_ptr, d.crecv_p, d.cl_rank, d.cl_coef,
                                                             (const TV*)d.cpart, Yh);
                end(7);
            } else {
                k_coupling<TB, TV><<<d.n_rowcl, 256, 0, s>>>(d.row_cl, d.row_ncols, d.row_off, d.row_colptr,
                                                             d.colsrc, d.cl_rank, d.cl_coef, coupling, Xh, Yh);
                end(3);
            }
            begin(4);
            for (int l = 0; l < lv.n_down; ++l)
                if (lv.down_count[l] > 0)
                    k_transfer_down<TB, TV><<<lv.down_count[l], 64, 0, s>>>(d.down_list + lv.down_begin[l], d.cl_rank,
                                                                            d.cl_coef, d.cl_parent, d.cl_transfer_off,
                                                                            transfer, Yh);
            end(4);
        }
        if (overlap) {                   // the last pass waits for the side stream's passes
            hipError_t e = hipStreamWaitEvent(s, d.near_join, 0);
            if (e != hipSuccess) return e;
        }
        begin(5);
        if (d.near_sym) {
            auto kn = d.near_cached ? k_near_sym<TB, TV, false> : k_near_sym<TB, TV, true>;
            kn<<<d.n_leaves, 256, 0, s>>>(d.sym_leaf, d.sym_ptr, d.sym_sbeg, d.sym_ssize, d.sym_off, d.sym_pslot, near,
                                          d.cl_begin, d.cl_size, U, (TV*)d.sym_rows, (TV*)d.sym_part);
            end(5);
            begin(6);
            k_near_sym_finish<TB, TV><<<d.n_leaves, 64, 0, s>>>(d.sym_leaf, d.sym_in_ptr, d.sym_in_slot,
                                                                (const TV*)d.sym_rows, (const TV*)d.sym_part, d.cl_rank,
                                                                d.cl_coef, d.cl_begin, d.cl_size, d.cl_basis_off, basis,
                                                                Yh, d.perm, xr, yr, op, alpha);
            end(6);
        } else if (tiles) {
            near_tile(overlap ? 1 : 2, xr, yr, s);
            end(5);
        } else if (overlap) {
            near_pass(d.near_passes - 1, xr, yr, s);
            end(5);
        } else {
            for (int pass = 0; pass < d.near_passes; ++pass) near_pass(pass, xr, yr, s);
            end(5);
        }
    }
    return hipGetLastError();
}

hipError_t launch_matvec(const DevH2& d, const LevelLaunch& lv, int op, int prec, const void* x, void* y,
                         int64_t n_rhs, int64_t ld, hipStream_t s, Profiler* prof) {
    if (prec == 0)
        return matvec_tier<double2, double2>(d, lv, op, d.tier[0], (const double2*)x, (double2*)y, n_rhs, ld, s, prof);
    if (prec == 1)
        return matvec_tier<float2, float2>(d, lv, op, d.tier[1], (const float2*)x, (float2*)y, n_rhs, ld, s, prof);
    return hipErrorInvalidValue;
}

}  // namespace h2
