// Batched (many right-hand sides, many geometries) BF16x3 tier: internal layout.
//
// Every block product of the H^2 product (near blocks, couplings, leaf bases,
// transfers) becomes a complex block GEMM C (M x W) (+)= A (M x K) B (K x W)
// over W = 3 * n_rhs columns, done in real arithmetic on the matrix cores:
//   [Cr; Ci] = [Ar -Ai; Ai Ar] [Br; Bi],
// each real operand split into bf16 hi + lo parts and multiplied as
// hi*hi + hi*lo + lo*hi with FP32 accumulation (v_mfma_f32_16x16x32_bf16).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace h2 {

// One output row block (its rows padded to a multiple of 16).
struct BOwner {
    float* out;        // FP32 output planes: re plane at out, im plane at out + ps; row 0 of this owner
    int64_t ld;        // rows per column of the output planes
    int64_t ps;        // plane stride (elements)
    int mp;            // padded complex rows (multiple of 16, <= 64)
    int t0, nt;        // terms [t0, t0 + nt)
    int acc;           // 1: add to the existing output
};

// One A (M x K) block times the B rows of one source.
struct BTerm {
    const uint16_t* a;  // A planes: Ar_hi, Ar_lo, Ai_hi, Ai_lo, each mp x kp bf16 row major
    const uint16_t* b;  // B planes (re_hi, re_lo, im_hi, im_lo) at the source's first row
    int64_t bld;        // rows per column of the B planes
    int64_t bps;        // plane stride of the B planes (elements)
    int kp;             // padded complex K (multiple of 16, <= 64)
    int pad;
};

// Conversion of FP32 planes rows [r0, r0 + nrows) into bf16 hi/lo planes.
struct SplitSeg {
    const float* src;   // re plane (im at src + sps)
    int64_t sld, sps;
    uint16_t* dst;      // re_hi plane (re_lo, im_hi, im_lo at dst + q * dps)
    int64_t dld, dps;
    int r0, nrows;
};

// A block packing job: source complex block (col major, M x K, or its transpose)
// into the four bf16 planes of an A operand.
struct PackJob {
    int64_t src;        // complex offset in the FP64 source array
    int64_t dst;        // bf16 element offset in the arena
    int m, k, mp, kp;   // logical and padded sizes of A
    int src_rows;       // leading dimension of the source (col major)
    int transpose;      // 1: A = source^T
    int which;          // 0 near, 1 coupling, 2 basis, 3 transfer
    int pad;
};

// Relative (offset) form of a phase, built at plan time.
struct RelOwner { int out_kind; int64_t out_row; int mp, t0, nt, acc; };      // out_kind: 0 Xf, 1 Yhat f, 2 Yf
struct RelTerm { int64_t a; int b_kind; int64_t b_row; int kp; };             // b_kind: 0 U, 1 Xb, 2 Yhat b
struct RelPhase {
    std::vector<RelOwner> owners;
    std::vector<RelTerm> terms;
    int split_kind = -1;            // -1 none, 0: X planes, 1: Yhat planes
    int64_t split_r0 = 0, split_rows = 0;
};

// Everything one handle contributes to batched products.
struct BatchHost {
    int max_cols = 0;               // 3 * max_rhs
    int64_t urows = 0, crows = 0;   // padded rows of the voxel and coefficient planes
    int n_leaf_phase = 1;
    std::vector<RelPhase> up, down; // per level step (deepest parents first / top children first)
    RelPhase leaf, coup, near;
    std::vector<PackJob> jobs;
    std::vector<int> prow;          // padded row of each tree position
    int64_t arena_elems = 0;        // bf16 elements
    // device addresses (set at build)
    uint16_t* arena = nullptr;
    uint16_t *Ub = nullptr, *Xb = nullptr, *Yhb = nullptr;
    float *Xf = nullptr, *Yhf = nullptr, *Yf = nullptr;
    int* prow_dev = nullptr;
};

// Absolute (device pointer) phase of a group, concatenated over members.
struct GPhase {
    std::vector<BOwner> owners;
    std::vector<BTerm> terms;
    std::vector<SplitSeg> splits;   // run after the GEMM
    std::vector<int> owner_member;  // member of each owner (column count)
};

// kernels (h2_batch.hip)
hipError_t launch_pack(const PackJob* jobs_dev, int njobs, const double2* const* srcs, uint16_t* arena,
                       hipStream_t s);
hipError_t launch_fill_u16(uint16_t* p, int64_t n, hipStream_t s);
// plane = elements per plane (rows x allocated columns)
hipError_t launch_prologue_b(int n_vox, const int* perm, const int* prow, const double2* chi, const float2* x,
                             int64_t ldx, int ncols, uint16_t* Ub, int64_t urows, int64_t plane, int op, hipStream_t s);
hipError_t launch_split(const SplitSeg* segs, int nseg, int max_elems_per_seg, const int* seg_cols, hipStream_t s);
hipError_t launch_bgemm(int nc, const BOwner* owners, const BTerm* terms, const int2* tasks, int ntasks,
                        const int* owner_cols, hipStream_t s);
hipError_t launch_epilogue_b(int n_vox, const int* perm, const int* prow, const float* Yf, int64_t urows,
                             int64_t plane, const float2* x, int64_t ldx, float2* y, int64_t ldy, int ncols, int op,
                             float alpha, hipStream_t s);

}  // namespace h2
