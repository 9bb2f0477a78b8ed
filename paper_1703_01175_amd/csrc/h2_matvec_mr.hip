// H^2 product on several right-hand sides per pass (FP64 / FP32 tiers).
//
// The same sequence as the single-vector product of Sec. IV.B (prologue, leaf
// forward, upward transfers, couplings, downward transfers, near field + leaf
// backward + epilogue), with kMrRhs right-hand sides (kMrCols = 3 kMrRhs
// columns) carried through every pass: each block element read from memory is
// used for kMrCols complex FMAs instead of 3, which moves the near field from
// 1.5 to 6 flop per byte (FP64), still under the ridge of the vector units.
// Vectors in tree order are [row][kMrCols]; columns 3 r + c hold component c of
// right-hand side r of the pass (zero beyond the pass's right-hand sides).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "h2_internal.h"

namespace h2 {
namespace {

template <typename TV> struct RealOf;
template <> struct RealOf<double2> { using T = double; };
template <> struct RealOf<float2> { using T = float; };

template <typename TV, typename TB>
__device__ __forceinline__ void mr_fma(TV& acc, TB a, TV b) {
    using R = typename RealOf<TV>::T;
    const R ax = (R)a.x, ay = (R)a.y;
    acc.x = fma(ax, b.x, acc.x);
    acc.x = fma(-ay, b.y, acc.x);
    acc.y = fma(ax, b.y, acc.y);
    acc.y = fma(ay, b.x, acc.y);
}

template <typename TV> __device__ __forceinline__ TV mr_zero() { TV z; z.x = 0; z.y = 0; return z; }
template <typename TV> __device__ __forceinline__ TV mr_add(TV a, TV b) { TV r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }

__device__ __forceinline__ double2 mr_ldnt(const double2* p) {
    return make_double2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}
__device__ __forceinline__ float2 mr_ldnt(const float2* p) {
    return make_float2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}

// near-block loads: streaming when each block is read once, cached when identical
// blocks are stored once and reread
template <bool NT, typename T> __device__ __forceinline__ T mr_ldblk(const T* p) {
    if constexpr (NT) return mr_ldnt(p);
    else return *p;
}

constexpr int C = kMrCols;

// U[p][3 r + c] = chi[v] x_r[3 v + c] (op Z) or x_r[3 v + c] (op G), v = perm[p]; 0 for r >= nr
template <typename TV>
__global__ void k_prologue_mr(int n_vox, const int* __restrict__ perm, const double2* __restrict__ chi,
                              const TV* __restrict__ x, int64_t ld, int nr, TV* __restrict__ U, int op) {
    using R = typename RealOf<TV>::T;
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < (int64_t)n_vox * C;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int p = int(e / C), col = int(e % C);
        const int r = col / 3, c = col % 3;
        TV o = mr_zero<TV>();
        if (r < nr) {
            const int v = perm[p];
            const TV a = x[r * ld + (int64_t)v * 3 + c];
            if (op == 1) {
                const R cr = (R)chi[v].x, ci = (R)chi[v].y;
                o.x = cr * a.x - ci * a.y;
                o.y = cr * a.y + ci * a.x;
            } else {
                o = a;
            }
        }
        U[e] = o;
    }
}

// X_t[a][col] = sum_i V_t[i, a] U_t[i][col]; one group per leaf, U_t staged in LDS
template <typename TB, typename TV>
__global__ __launch_bounds__(256) void k_leaf_forward_mr(const int* __restrict__ leaf_id, const int* __restrict__ cl_rank,
                                                         const int* __restrict__ cl_coef, const int* __restrict__ cl_begin,
                                                         const int* __restrict__ cl_size,
                                                         const int64_t* __restrict__ cl_basis_off,
                                                         const TB* __restrict__ basis, const TV* __restrict__ U,
                                                         TV* __restrict__ Xh) {
    __shared__ TV su[kMaxLeaf * C];
    const int t = leaf_id[blockIdx.x];
    const int k = cl_rank[t];
    if (k == 0) return;                       // uniform over the group, before the barrier
    const int n = cl_size[t];
    const int b0 = cl_begin[t];
    for (int e = threadIdx.x; e < n * C; e += 256) su[e] = U[(int64_t)b0 * C + e];
    __syncthreads();
    const TB* V = basis + cl_basis_off[t];
    const int co = cl_coef[t];
    for (int e = threadIdx.x; e < k * C; e += 256) {
        const int a = e / C, col = e % C;
        TV acc = mr_zero<TV>();
        const TB* vc = V + (int64_t)a * n;
        for (int i = 0; i < n; ++i) mr_fma(acc, vc[i], su[i * C + col]);
        Xh[(int64_t)(co + a) * C + col] = acc;
    }
}

// X_p[a][col] = sum_children sum_b T_c[b, a] X_c[b][col]
template <typename TB, typename TV>
__global__ __launch_bounds__(256) void k_transfer_up_mr(const int* __restrict__ list, const int* __restrict__ cl_rank,
                                                        const int* __restrict__ cl_coef,
                                                        const int* __restrict__ cl_first_child,
                                                        const int* __restrict__ cl_nchild,
                                                        const int64_t* __restrict__ cl_toff,
                                                        const TB* __restrict__ transfer, TV* __restrict__ Xh) {
    const int p = list[blockIdx.x];
    const int kp = cl_rank[p];
    const int c0 = cl_first_child[p], nc = cl_nchild[p];
    for (int e = threadIdx.x; e < kp * C; e += 256) {
        const int a = e / C, col = e % C;
        TV acc = mr_zero<TV>();
        for (int ch = c0; ch < c0 + nc; ++ch) {
            const int kc = cl_rank[ch];
            if (kc == 0) continue;
            const TB* T = transfer + cl_toff[ch] + (int64_t)a * kc;
            const TV* xc = Xh + (int64_t)cl_coef[ch] * C + col;
            for (int b = 0; b < kc; ++b) mr_fma(acc, T[b], xc[(int64_t)b * C]);
        }
        Xh[(int64_t)(cl_coef[p] + a) * C + col] = acc;
    }
}

// Y_t = [S_ts1 S_ts2 ...] gather(X): the gathered coefficient rows of a chunk of
// kChunk grouped columns are staged in LDS; lanes are RW rows x (64 / RW) column
// streams, and the 4 (64 / RW) streams of the group split the chunk's columns, so
// every element of S is loaded once and used for all kMrCols columns.  The
// streams' partial rows are summed through LDS three columns at a time.
constexpr int kChunk = 64;

template <typename TB, typename TV, int RW>
__device__ __forceinline__ void coupling_mr_rows(int kt, int ncols, const TB* __restrict__ S,
                                                 const int* __restrict__ src, const TV* __restrict__ Xh,
                                                 TV* __restrict__ Yh, int co, TV (*xs)[C], TV (*red)[3]) {
    constexpr int G = 64 / RW;               // streams per wave
    constexpr int NS = 4 * G;                // streams per group
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int a = lane % RW;
    const int sid = w * G + lane / RW;       // this lane's column stream
    for (int r0 = 0; r0 < kt; r0 += RW) {
        const int row = r0 + a;
        const bool live = row < kt;
        TV acc[C];
#pragma unroll
        for (int q = 0; q < C; ++q) acc[q] = mr_zero<TV>();
        for (int j0 = 0; j0 < ncols; j0 += kChunk) {
            const int nj = min(kChunk, ncols - j0);
            __syncthreads();                 // the previous chunk is no longer read
            for (int e = threadIdx.x; e < nj * C; e += 256) {
                const int jj = e / C, q = e % C;
                xs[jj][q] = Xh[(int64_t)src[j0 + jj] * C + q];
            }
            __syncthreads();
            if (live)
                for (int jj = sid; jj < nj; jj += NS) {
                    const TB sv = mr_ldnt(S + (int64_t)(j0 + jj) * kt + row);
#pragma unroll
                    for (int q = 0; q < C; ++q) mr_fma(acc[q], sv, xs[jj][q]);
                }
        }
#pragma unroll
        for (int q0 = 0; q0 < C; q0 += 3) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 3; ++q) red[threadIdx.x][q] = acc[q0 + q];
            __syncthreads();
            // thread (row a, column q) sums the NS streams of that row
            if (threadIdx.x < RW * 3) {
                const int ra = threadIdx.x / 3, q = threadIdx.x % 3;
                if (r0 + ra < kt) {
                    TV sum = mr_zero<TV>();
                    for (int st = 0; st < NS; ++st) {
                        const int lt = (st / G) * 64 + (st % G) * RW + ra;   // thread of stream st, row ra
                        sum = mr_add(sum, red[lt][q]);
                    }
                    Yh[(int64_t)(co + r0 + ra) * C + q0 + q] = sum;
                }
            }
        }
    }
}

// FP64: the grouped row on the matrix cores (v_mfma_f64_16x16x4f64, complex products
// in the 3M form).  One group of four waves per row slot; wave w takes k steps w, w + 4,
// ... of 4 grouped columns each.  A = RT tiles of 16 rows x the step's 4 columns of S
// (lane l: row l % 16, column l / 16); B = the 4 columns' gathered coefficient rows x 16
// (lane l: column l / 16, right-hand-side column l % 16, zero past kMrCols).  Operands
// run two steps ahead, the gather indices three, each from a register ring reloaded
// right after its use; columns past the row's end read a zero entry instead of
// branching.  The four waves' sums meet in LDS (fixed order).
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int RT>
__device__ __forceinline__ void coupling_mr_mfma_rows(int kt, int ncols, const double2* __restrict__ S,
                                                      const int* __restrict__ src, const double2* __restrict__ Xh,
                                                      const double2* __restrict__ zero, double2* __restrict__ Yh,
                                                      int co, double2 (*red)[kMaxLeaf][16]) {
    constexpr int D = 2;                     // k steps of loads in flight per wave
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int rl = lane & 15, kq = lane >> 4;
    const int nsteps = (ncols + 3) >> 2;
    v4d acc[RT][3];
#pragma unroll
    for (int u = 0; u < RT; ++u)
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[u][q] = v4d{0, 0, 0, 0};
    struct Ops {
        double2 a[RT];
        double2 b;
    };
    // gather index of this lane's column in step i of this wave (its first column if past the end)
    auto gidx = [&](int i) {
        const int j = 4 * (w + 4 * i) + kq;
        return src[j < ncols ? j : 0];
    };
    auto load = [&](int i, int g) {
        const int j = 4 * (w + 4 * i) + kq;
        const bool ok = j < ncols;
        Ops o;
#pragma unroll
        for (int u = 0; u < RT; ++u) {
            const int r = 16 * u + rl;
            o.a[u] = *(ok && r < kt ? S + (int64_t)j * kt + r : zero);
        }
        o.b = *(ok && rl < C ? Xh + (int64_t)g * C + rl : zero);
        return o;
    };
    auto mma = [&](const Ops& o) {
        const double sb = o.b.x + o.b.y;
#pragma unroll
        for (int u = 0; u < RT; ++u) {
            acc[u][0] = mfma64(o.a[u].x, o.b.x, acc[u][0]);
            acc[u][1] = mfma64(o.a[u].y, o.b.y, acc[u][1]);
            acc[u][2] = mfma64(o.a[u].x + o.a[u].y, sb, acc[u][2]);
        }
    };
    const int mine = nsteps > w ? (nsteps - 1 - w) / 4 + 1 : 0;      // this wave's steps
    if (mine > 0) {
        // ring of D steps' operands and gather indices: slot u holds step i + u; each is
        // reloaded (D steps ahead) right after its use, past the end with zeros
        Ops ops[D];
        int g[D];
#pragma unroll
        for (int u = 0; u < D; ++u) g[u] = gidx(u);
#pragma unroll
        for (int u = 0; u < D; ++u) ops[u] = load(u, g[u]);
#pragma unroll
        for (int u = 0; u < D; ++u) g[u] = gidx(u + D);
        for (int i = 0; i < mine; i += D) {
#pragma unroll
            for (int u = 0; u < D; ++u) {
                mma(ops[u]);
                ops[u] = load(i + u + D, g[u]);
                g[u] = gidx(i + u + 2 * D);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    // register r of lane l in tile u: row 16 u + 4 r + l / 16, column l % 16
#pragma unroll
    for (int u = 0; u < RT; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            red[w][16 * u + 4 * r + kq][rl] =
                make_double2(acc[u][0][r] - acc[u][1][r], acc[u][2][r] - acc[u][0][r] - acc[u][1][r]);
    __syncthreads();
    for (int e = threadIdx.x; e < kt * C; e += 256) {
        const int r = e / C, c = e % C;
        double2 sum = red[0][r][c];
        sum = mr_add(sum, red[1][r][c]);
        sum = mr_add(sum, red[2][r][c]);
        sum = mr_add(sum, red[3][r][c]);
        Yh[(int64_t)(co + r) * C + c] = sum;
    }
}

__global__ __launch_bounds__(256) void k_coupling_mr_mfma(const int* __restrict__ row_cl,
                                                          const int* __restrict__ row_ncols,
                                                          const int64_t* __restrict__ row_off,
                                                          const int* __restrict__ row_colptr,
                                                          const int* __restrict__ colsrc,
                                                          const int* __restrict__ cl_rank,
                                                          const int* __restrict__ cl_coef,
                                                          const double2* __restrict__ coupling,
                                                          const double2* __restrict__ zero,
                                                          const double2* __restrict__ Xh, double2* __restrict__ Yh) {
    __shared__ double2 red[4][kMaxLeaf][16];
    const int slot = blockIdx.x;
    const int t = row_cl[slot];
    const int kt = cl_rank[t];
    const int ncols = row_ncols[slot];
    const double2* S = coupling + row_off[slot];
    const int* src = colsrc + row_colptr[slot];
    const int co = cl_coef[t];
    if (kt <= 16)
        coupling_mr_mfma_rows<1>(kt, ncols, S, src, Xh, zero, Yh, co, red);
    else if (kt <= 32)
        coupling_mr_mfma_rows<2>(kt, ncols, S, src, Xh, zero, Yh, co, red);
    else
        coupling_mr_mfma_rows<4>(kt, ncols, S, src, Xh, zero, Yh, co, red);
}

template <typename TB, typename TV>
__global__ __launch_bounds__(256) void k_coupling_mr(const int* __restrict__ row_cl, const int* __restrict__ row_ncols,
                                                     const int64_t* __restrict__ row_off,
                                                     const int* __restrict__ row_colptr, const int* __restrict__ colsrc,
                                                     const int* __restrict__ cl_rank, const int* __restrict__ cl_coef,
                                                     const TB* __restrict__ coupling, const TV* __restrict__ Xh,
                                                     TV* __restrict__ Yh) {
    __shared__ TV xs[kChunk][C];
    __shared__ TV red[256][3];
    const int slot = blockIdx.x;
    const int t = row_cl[slot];
    const int kt = cl_rank[t];
    const int ncols = row_ncols[slot];
    const TB* S = coupling + row_off[slot];
    const int* src = colsrc + row_colptr[slot];
    const int co = cl_coef[t];
    if (kt <= 16)
        coupling_mr_rows<TB, TV, 16>(kt, ncols, S, src, Xh, Yh, co, xs, red);
    else if (kt <= 32)
        coupling_mr_rows<TB, TV, 32>(kt, ncols, S, src, Xh, Yh, co, xs, red);
    else
        coupling_mr_rows<TB, TV, 64>(kt, ncols, S, src, Xh, Yh, co, xs, red);
}

// Y_c[b][col] += sum_a T_c[b, a] Y_p[a][col]
template <typename TB, typename TV>
__global__ __launch_bounds__(256) void k_transfer_down_mr(const int* __restrict__ list, const int* __restrict__ cl_rank,
                                                          const int* __restrict__ cl_coef,
                                                          const int* __restrict__ cl_parent,
                                                          const int64_t* __restrict__ cl_toff,
                                                          const TB* __restrict__ transfer, TV* __restrict__ Yh) {
    const int ch = list[blockIdx.x];
    const int p = cl_parent[ch];
    const int kc = cl_rank[ch], kp = cl_rank[p];
    const TB* T = transfer + cl_toff[ch];
    const TV* yp = Yh + (int64_t)cl_coef[p] * C;
    for (int e = threadIdx.x; e < kc * C; e += 256) {
        const int b = e / C, col = e % C;
        TV acc = mr_zero<TV>();
        for (int a = 0; a < kp; ++a) mr_fma(acc, T[(int64_t)a * kc + b], yp[(int64_t)a * C + col]);
        TV* o = Yh + (int64_t)(cl_coef[ch] + b) * C + col;
        *o = mr_add(*o, acc);
    }
}

// Near field + leaf backward + epilogue: one group per leaf, wave w streams blocks
// w, w + 4, ...; lane i owns row i; the source values U_s[j][col] are wave-uniform.
template <typename TB, typename TV, bool NT>
__global__ __launch_bounds__(256) void k_near_epilogue_mr(
    const int* __restrict__ leaf_id, const int* __restrict__ near_ptr, const int* __restrict__ near_sbeg,
    const int* __restrict__ near_ssize, const int64_t* __restrict__ near_off, const TB* __restrict__ near,
    const int* __restrict__ cl_rank, const int* __restrict__ cl_coef, const int* __restrict__ cl_begin,
    const int* __restrict__ cl_size, const int64_t* __restrict__ cl_basis_off, const TB* __restrict__ basis,
    const TV* __restrict__ U, const TV* __restrict__ Yh, const int* __restrict__ perm, const TV* __restrict__ x,
    TV* __restrict__ y, int64_t ld, int nr, int op, typename RealOf<TV>::T alpha) {
    __shared__ TV red[4][kMaxLeaf][3];
    const int slot = blockIdx.x;
    const int t = leaf_id[slot];
    const int n = cl_size[t];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    TV acc[C];
#pragma unroll
    for (int q = 0; q < C; ++q) acc[q] = mr_zero<TV>();
    const int e = near_ptr[slot + 1];
    for (int blk = near_ptr[slot] + w; blk < e; blk += 4) {
        const int sb = near_sbeg[blk];
        const int ns = near_ssize[blk];
        const TB* Gb = near + near_off[blk] + lane;
        const TV* us = U + (int64_t)sb * C;
        if (lane < n) {
#pragma unroll 2
            for (int j = 0; j < ns; ++j) {
                const TB gv = mr_ldblk<NT>(Gb + (int64_t)j * n);
#pragma unroll
                for (int q = 0; q < C; ++q) mr_fma(acc[q], gv, us[j * C + q]);
            }
        }
    }
    // sum the four waves' rows, three columns at a time; wave 0 keeps the sums
#pragma unroll
    for (int q0 = 0; q0 < C; q0 += 3) {
#pragma unroll
        for (int q = 0; q < 3; ++q) red[w][lane][q] = acc[q0 + q];
        __syncthreads();
        if (w == 0)
#pragma unroll
            for (int q = 0; q < 3; ++q)
                acc[q0 + q] = mr_add(mr_add(red[0][lane][q], red[1][lane][q]), mr_add(red[2][lane][q], red[3][lane][q]));
        __syncthreads();
    }
    if (w != 0 || lane >= n) return;
    const int k = cl_rank[t];
    if (k > 0) {   // backward transformation at the leaf: y_t += V_t Y_t
        const TB* V = basis + cl_basis_off[t];
        const TV* yt = Yh + (int64_t)cl_coef[t] * C;
        for (int a = 0; a < k; ++a) {
            const TB v = V[(int64_t)a * n + lane];
#pragma unroll
            for (int q = 0; q < C; ++q) mr_fma(acc[q], v, yt[(int64_t)a * C + q]);
        }
    }
    const int64_t vox = perm[cl_begin[t] + lane];
#pragma unroll
    for (int q = 0; q < C; ++q) {
        const int r = q / 3, c = q % 3;
        if (r >= nr) break;
        const int64_t o = r * ld + vox * 3 + c;
        TV out = acc[q];
        if (op == 1) {
            out.x = x[o].x + alpha * acc[q].x;
            out.y = x[o].y + alpha * acc[q].y;
        }
        y[o] = out;
    }
}

template <typename TB, typename TV>
hipError_t mr_tier(const DevH2& d, const LevelLaunch& lv, int op, const TierData& td, const TV* x, TV* y,
                   int64_t n_rhs, int64_t ld, hipStream_t s) {
    using R = typename RealOf<TV>::T;
    const TB* near = (const TB*)td.near;
    const TB* coupling = (const TB*)td.coupling;
    const TB* basis = (const TB*)td.basis;
    const TB* transfer = (const TB*)td.transfer;
    TV* U = (TV*)d.U;
    TV* Xh = (TV*)d.Xh;
    TV* Yh = (TV*)d.Yh;
    const R alpha = (R)(d.sigma * d.k * d.k * d.volume);
    const int pro_grid = int(std::min<int64_t>(((int64_t)d.n_vox * C + 255) / 256, 65536));
    for (int64_t r0 = 0; r0 < n_rhs; r0 += kMrRhs) {
        const int nr = int(std::min<int64_t>(kMrRhs, n_rhs - r0));
        const TV* xr = x + r0 * ld;
        TV* yr = y + r0 * ld;
        k_prologue_mr<TV><<<pro_grid, 256, 0, s>>>(d.n_vox, d.perm, d.chi, xr, ld, nr, U, op);
        if (d.coef_rows > 0) {
            k_leaf_forward_mr<TB, TV><<<d.n_leaves, 256, 0, s>>>(d.leaf_id, d.cl_rank, d.cl_coef, d.cl_begin,
                                                                 d.cl_size, d.cl_basis_off, basis, U, Xh);
            for (int l = 0; l < lv.n_up; ++l)
                if (lv.up_count[l] > 0)
                    k_transfer_up_mr<TB, TV><<<lv.up_count[l], 256, 0, s>>>(d.up_list + lv.up_begin[l], d.cl_rank,
                                                                            d.cl_coef, d.cl_first_child, d.cl_nchild,
                                                                            d.cl_transfer_off, transfer, Xh);
            // FP64 with ranks up to 64: on the matrix cores
            bool done = false;
            if constexpr (std::is_same<TV, double2>::value && std::is_same<TB, double2>::value) {
                if (d.coupling_mr_mfma) {
                    k_coupling_mr_mfma<<<d.n_rowcl, 256, 0, s>>>(d.row_cl, d.row_ncols, d.row_off, d.row_colptr,
                                                                 d.colsrc, d.cl_rank, d.cl_coef, coupling,
                                                                 (const double2*)d.zero_block, Xh, Yh);
                    done = true;
                }
            }
            if (!done)
                k_coupling_mr<TB, TV><<<d.n_rowcl, 256, 0, s>>>(d.row_cl, d.row_ncols, d.row_off, d.row_colptr,
                                                                d.colsrc, d.cl_rank, d.cl_coef, coupling, Xh, Yh);
            for (int l = 0; l < lv.n_down; ++l)
                if (lv.down_count[l] > 0)
                    k_transfer_down_mr<TB, TV><<<lv.down_count[l], 256, 0, s>>>(d.down_list + lv.down_begin[l],
                                                                                d.cl_rank, d.cl_coef, d.cl_parent,
                                                                                d.cl_transfer_off, transfer, Yh);
        }
        auto kn = d.near_cached ? k_near_epilogue_mr<TB, TV, false> : k_near_epilogue_mr<TB, TV, true>;
        kn<<<d.n_leaves, 256, 0, s>>>(d.leaf_id, d.near_ptr, d.near_sbeg, d.near_ssize, d.near_off, near, d.cl_rank,
                                      d.cl_coef, d.cl_begin, d.cl_size, d.cl_basis_off, basis, U, Yh, d.perm, xr, yr,
                                      ld, nr, op, alpha);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_matvec_multi(const DevH2& d, const LevelLaunch& lv, int op, int prec, const void* x, void* y,
                               int64_t n_rhs, int64_t ld, hipStream_t s) {
    if (n_rhs < 2 || d.vec_cols < kMrCols) return launch_matvec(d, lv, op, prec, x, y, n_rhs, ld, s);
    if (prec == 0)
        return mr_tier<double2, double2>(d, lv, op, d.tier[0], (const double2*)x, (double2*)y, n_rhs, ld, s);
    if (prec == 1)
        return mr_tier<float2, float2>(d, lv, op, d.tier[1], (const float2*)x, (float2*)y, n_rhs, ld, s);
    return hipErrorInvalidValue;
}

}  // namespace h2
