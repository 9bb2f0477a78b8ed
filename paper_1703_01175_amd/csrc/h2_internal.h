// Internal layout shared by the host packer (h2vie_api.cpp) and the HIP
// kernels (h2_matvec.hip, h2_krylov.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace h2 {

constexpr int kNcomp = 3;        // field components per voxel
constexpr int kMaxLeaf = 64;     // voxels per leaf cluster
constexpr int kTileLeaves = 16;  // target leaves per tile of the tiled near field
constexpr int kMrRhs = 4;        // right-hand sides per pass of the multi-RHS FP64 / FP32 product
constexpr int kMrCols = kNcomp * kMrRhs;
constexpr int kMaxRank = 256;    // cluster rank limit
constexpr int64_t kNearPassBytes = int64_t(2) << 20;   // distinct near-block bytes per near-field pass

// Storage tier of the block data (near blocks, couplings, bases, transfers).
struct TierData {
    const void* near = nullptr;      // per near block, #t x #s column major
    const void* coupling = nullptr;  // grouped block rows, k_t x sum(k_s) column major
    const void* basis = nullptr;     // leaf bases, #t x k_t column major
    const void* transfer = nullptr;  // T_c, k_c x k_parent column major
    // BF16 hi+lo tier: low parts (same layout as the hi arrays above)
    const void* near_lo = nullptr;
    const void* coupling_lo = nullptr;
    const void* basis_lo = nullptr;
    const void* transfer_lo = nullptr;
};

// Leaves in cluster order, for the per-leaf preconditioners.
struct LeafInfo {
    int n = 0;                        // number of leaves
    const int* beg = nullptr;         // first tree position
    const int* size = nullptr;        // voxels
    const int64_t* diag = nullptr;    // complex offset of the diagonal near block G_tt
    const int64_t* inv_off = nullptr; // complex offset of [M_t | I] in the block-diagonal buffer
    int64_t inv_elems = 0;            // total complex elements of that buffer
    int max_leaf = 0;
};

// Everything a product needs, as device pointers into the caller's buffer.
struct DevH2 {
    int n_vox = 0;
    int n_clusters = 0;
    int n_leaves = 0;
    int coef_rows = 0;          // sum of ranks
    int n_rowcl = 0;            // row clusters of the coupling launch (rank > 0)
    int depth = 0;
    double k = 0, volume = 0, sigma = 1;

    const int* perm = nullptr;          // [n_vox] tree position -> voxel
    const double2* chi = nullptr;       // [n_vox] caller order

    // clusters
    const int* cl_rank = nullptr;
    const int* cl_coef = nullptr;       // first coefficient row
    const int* cl_begin = nullptr;
    const int* cl_size = nullptr;
    const int* cl_parent = nullptr;
    const int* cl_first_child = nullptr;
    const int* cl_nchild = nullptr;
    const int64_t* cl_transfer_off = nullptr;  // complex offset of T_c (-1 none)
    const int64_t* cl_basis_off = nullptr;     // complex offset of V_c (-1 none)

    // leaves in launch order (most near blocks first)
    const int* leaf_id = nullptr;       // [n_leaves]
    const int* near_ptr = nullptr;      // [n_leaves + 1] into the near block list
    const int* near_sbeg = nullptr;     // per near block: tree position of s
    const int* near_ssize = nullptr;    // per near block: #s
    const int64_t* near_off = nullptr;  // per near block: complex offset of G_ts

    // coupling launch (row clusters, most work first)
    const int* row_cl = nullptr;        // [n_rowcl]
    bool coupling_mr_mfma = false;      // ranks <= 64: multi-RHS FP64 couplings on the matrix cores
    const int* row_ncols = nullptr;     // grouped columns sum(k_s)
    const int64_t* row_off = nullptr;   // complex offset of the grouped block row
    const int* row_colptr = nullptr;    // first entry in colsrc
    const int* colsrc = nullptr;        // coefficient row of each grouped column

    // symmetric couplings (S_st = S_ts^T for every pair): each unordered pair streamed
    // once by its owner, which also writes S_ts^T X_t for the other cluster
    bool coup_sym_ok = false;           // the description's couplings allow it
    bool coup_sym = false;              // single-vector FP64 / FP32 products use it
    const int* row_nown = nullptr;      // per row slot: owned columns (stored first in the row)
    const int* row_pbase = nullptr;     // per row slot: its first partial column
    const int* crecv_ptr = nullptr;     // [n_rowcl + 1] into crecv_p
    const int* crecv_p = nullptr;       // partial column of the first column of each received block
    void* cpart = nullptr;              // [owned columns][3] partials S_ts^T X_t (vector type)

    // per-level lists for the upward / downward passes
    const int* up_list = nullptr;       // parents with rank > 0, grouped by level (deepest first)
    const int* down_list = nullptr;     // children with a transfer, grouped by level (top first)

    bool near_cached = false;           // identical near blocks stored once: read them through the caches
    int near_passes = 1;                // full-mode near launches, each over a share of the distinct blocks
    const int* near_pass_ptr = nullptr; // [n_leaves][near_passes + 1] list ranges of each pass
    void* near_ypart = nullptr;         // [n_vox][3] tree order: rows summed by the earlier passes
    // the earlier passes need only U: they run on a side stream while the product's
    // stream runs the upward pass, the couplings and the downward pass (unset: in order)
    hipStream_t near_side = nullptr;
    hipEvent_t near_fork = nullptr, near_join = nullptr;
    // tiled near field (FP64, stored-once blocks, full mode): tiles of kTileLeaves target
    // leaves; step q of a tile is one stored block and, per target slot, the tree position
    // of the source leaf it multiplies (-1: none)
    const void* zero_block = nullptr;   // [kMaxLeaf][3] zeros (FP64): read in place of absent operands
    bool near_tiles_ok = false;         // the plan has tiles (blocks stored once)
    bool near_tiles = false;            // FP64 full-mode products use them
    bool tiles_full = false;            // every step is a kMaxLeaf x kMaxLeaf block
    int n_tiles = 0;
    const int* tile_ptr = nullptr;      // [n_tiles + 1] into the step list
    const int* tile_leaf = nullptr;     // [n_tiles][kTileLeaves] target leaves (-1: none)
    const int64_t* step_off = nullptr;  // per step: complex offset of its stored block
    const int* step_shape = nullptr;    // per step: rows | columns << 16
    const int* step_src = nullptr;      // [steps][kTileLeaves] source tree positions (-1: none)
    void* tile_part1 = nullptr;         // [n_vox][3] tree order: the second split group's sums (FP64)
    // symmetric near field (each unordered leaf pair streamed once; see the plan)
    bool near_sym_ok = false;           // the description's near blocks satisfy G_st = G_ts^T
    bool near_sym = false;              // products use it (selectable while near_sym_ok)
    const int* sym_leaf = nullptr;      // [n_leaves] leaves in launch order (most owned blocks first)
    const int* sym_ptr = nullptr;       // [n_leaves + 1] into the owned block list (diagonal first)
    const int* sym_sbeg = nullptr;      // per owned block: tree position of the other leaf
    const int* sym_ssize = nullptr;     // per owned block: its size
    const int* sym_pslot = nullptr;     // per owned block: partial slot of G^T u_t (-1: diagonal)
    const int* sym_in_ptr = nullptr;    // [n_leaves + 1] into sym_in_slot, by launch slot
    const int* sym_in_slot = nullptr;   // partial slots that land in each leaf
    const int64_t* sym_off = nullptr;   // per owned block: complex offset of G_(owner, other)
    void* sym_part = nullptr;           // [pairs][kMaxLeaf][3] partials (vector type)
    void* sym_rows = nullptr;           // [n_vox][3] tree order: each leaf's own rows

    LeafInfo leaves;

    TierData tier[3];
    bool has_tier[3] = {true, false, false};

    // scratch for one product pass (vec_cols columns: 3, or kMrCols when built with max_rhs >= 2)
    int vec_cols = kNcomp;
    void* U = nullptr;                  // [n_vox][ncols] tree order, vector type
    void* Xh = nullptr;                 // [coef_rows][ncols]
    void* Yh = nullptr;                 // [coef_rows][ncols]
};

// Host-side copies of the per-level launch sizes.
struct LevelLaunch {
    int up_begin[64], up_count[64];     // per level step (deepest first)
    int down_begin[64], down_count[64]; // per level step (top first)
    int n_up = 0, n_down = 0;
};

// Optional per-family event recording around kernel launches.
struct Profiler {
    virtual ~Profiler() {}
    virtual void begin(int family, hipStream_t s) = 0;
    virtual void end(int family, hipStream_t s) = 0;
};

// Launchers (h2_matvec.hip).  ncols = 3 * n_rhs columns are processed as
// n_rhs passes of 3; x/y have leading dimension ld (complex elements).
hipError_t launch_matvec(const DevH2& d, const LevelLaunch& lv, int op, int prec, const void* x,
                         void* y, int64_t n_rhs, int64_t ld, hipStream_t s, Profiler* prof = nullptr);
// Several right-hand sides: passes of kMrRhs through the multi-RHS kernels
// (h2_matvec_mr.hip) when the scratch holds kMrCols columns, else launch_matvec.
hipError_t launch_matvec_multi(const DevH2& d, const LevelLaunch& lv, int op, int prec, const void* x, void* y,
                               int64_t n_rhs, int64_t ld, hipStream_t s);

}  // namespace h2
