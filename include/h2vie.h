/*
 * h2vie.h - C ABI of the MI355X H^2 volume-integral-equation hot path.
 *
 * The library applies, on one GPU, the minimal-rank H^2 representation of
 * the VIE system matrix (Omar & Jiao, Sec. III-IV) and solves the system
 * Z x = b with it (the paper's S D = E, eq. (2)):
 *
 *   Z x = x + sigma * k^2 * V * (G (x) I_ncomp) (chi . x),
 *
 * where G is the scalar Green's-function matrix between voxels held in H^2
 * form: dense near-field (inadmissible) leaf blocks, nested orthonormal
 * cluster bases (leaf bases V_t and transfer matrices T_c, eq. (9)) and one
 * coupling matrix S_ts per admissible block (eq. (8)).  The product follows
 * Sec. IV.B: forward transformation, coupling multiplication, backward
 * transformation, plus full products of the inadmissible blocks.
 *
 * Conventions for every entry point:
 *  - complex numbers are interleaved (re, im) doubles (FP64) unless a
 *    precision argument says otherwise; matrices are column major;
 *  - vectors live in device memory owned by the caller; unknown index
 *    ncomp*i + c for voxel i (caller's voxel order) and component c; a block
 *    of n_rhs vectors is column major with leading dimension ld >= N
 *    (N = ncomp * n_vox), in complex elements;
 *  - the stream argument is a hipStream_t passed as void* (NULL = null stream);
 *    every call is stream ordered and returns once its work is enqueued,
 *    except where a call says it synchronises;
 *  - no exception crosses the ABI: each call returns an h2_status, and
 *    h2_last_error() gives a thread-local message for the last failure;
 *  - inputs are never modified; a handle is used by one stream at a time.
 */
#ifndef H2VIE_H
#define H2VIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct h2_handle_s* h2_handle;

typedef enum {
    H2_OK = 0,
    H2_NOT_CONVERGED = 1,        /* warning: result written, tolerance not met */
    H2_ERR_INVALID_ARG = -1,     /* null/misaligned pointer, bad size, unknown enum */
    H2_ERR_BAD_DESC = -2,        /* host description inconsistent (indices, offsets, ranks) */
    H2_ERR_DEVICE = -3,          /* a HIP runtime call failed */
    H2_ERR_OOM = -4,             /* caller buffer smaller than the planned size */
    H2_ERR_BAD_HANDLE = -5,      /* null or destroyed handle */
    H2_ERR_NUMERIC = -6          /* NaN/Inf met in a solve */
} h2_status;

typedef enum { H2_FP64 = 0, H2_FP32 = 1, H2_BF16X3 = 2 } h2_precision;
typedef enum { H2_OP_G = 0, H2_OP_Z = 1 } h2_op;

/*
 * Host description of one H^2 representation (host memory, caller owned;
 * read during h2_plan_from_host / h2_build_from_host only).
 *
 * Clusters c = 0..n_clusters-1 are numbered breadth first (root = 0); each
 * owns the contiguous range [begin[c], end[c]) of tree positions, and
 * perm[p] is the caller's voxel index at tree position p (Sec. III.A).
 * rank[c] = k_c is the column count of the cluster basis (0 = unused).
 *  - leaf bases V_c (#c x k_c, col major) at basis + 2*basis_off[c]
 *    (basis_off = -1 for non-leaves or k_c = 0);
 *  - transfer T_c (k_c x k_parent, col major) at transfer + 2*transfer_off[c]
 *    (-1 where k_c or k_parent is 0);
 *  - far (admissible) pairs i: (far_t[i], far_s[i]) with S (k_t x k_s, col
 *    major) at coupling + 2*far_off[i].  All pairs of one row cluster t must be
 *    consecutive and their S blocks stored back to back, i.e. the grouped
 *    block row [S_ts1 S_ts2 ...] of t (eq. (5)) is one k_t x sum(k_s)
 *    column-major matrix;
 *  - near (inadmissible) pairs i: (near_t[i], near_s[i]), both leaves, with the
 *    dense block G_ts (#t x #s, col major) at near + 2*near_off[i]; pairs are
 *    sorted by near_t;
 *  - chi[2*n_vox]: complex contrast eps_r - 1 per voxel (caller order);
 *  - k (wavenumber), volume (voxel volume V), sigma (sign of the scattering
 *    term, +1 or -1).
 * Limits: ncomp == 3; leaf sizes <= 64; ranks <= 256; n_vox < 2^31.
 */
typedef struct {
    int64_t n_vox;
    int32_t ncomp;
    int32_t n_clusters;
    const int64_t* perm;
    const int32_t* level;
    const int32_t* parent;
    const int64_t* begin;
    const int64_t* end;
    const int32_t* first_child;
    const int32_t* nchild;
    const int32_t* rank;
    const int64_t* basis_off;
    const double* basis;
    int64_t basis_len;          /* complex elements */
    const int64_t* transfer_off;
    const double* transfer;
    int64_t transfer_len;
    int64_t n_far;
    const int32_t* far_t;
    const int32_t* far_s;
    const int64_t* far_off;
    const double* coupling;
    int64_t coupling_len;
    int64_t n_near;
    const int32_t* near_t;
    const int32_t* near_s;
    const int64_t* near_off;
    const double* near_blocks;
    int64_t near_len;
    const double* chi;
    double k;
    double volume;
    double sigma;
} h2_host_desc;

typedef struct {
    int32_t max_rhs;        /* most right-hand sides one call carries (>= 1) */
    int32_t tiers;          /* bit mask (1 << h2_precision) of storage tiers to hold;
                               FP64 is always held */
    int32_t flags;          /* H2_BUILD_* bits (0: defaults) */
    int32_t pad;
} h2_build_opts;

/* Near blocks that are identical bit for bit (same size and entries: on a uniform
 * voxel grid, every leaf pair of the same shape and relative position, since the
 * kernel depends on the offset between voxel centres only) are stored once on the
 * device and read through the caches, when that at least halves the near-block
 * storage; every block product is still carried out.  This flag keeps one stored
 * copy per near pair instead. */
#define H2_BUILD_KEEP_ALL_NEAR 1

/* Size (bytes) of the device buffer h2_build_from_host needs for d and o.
 * Validates d (same checks as the build).  Errors: INVALID_ARG, BAD_DESC. */
h2_status h2_plan_from_host(const h2_host_desc* d, const h2_build_opts* o, size_t* dev_bytes);

/* Validate d, pack it level by level into dev_buffer (caller-owned device
 * memory of at least the planned size, 256-byte aligned) and return a handle
 * that refers to that buffer.  Synchronises the stream before returning (the
 * host staging memory is released).  Errors: INVALID_ARG, BAD_DESC, OOM
 * (dev_bytes too small), DEVICE. */
h2_status h2_build_from_host(const h2_host_desc* d, const h2_build_opts* o, void* dev_buffer,
                             size_t dev_bytes, void* stream, h2_handle* out);

/* y = op(x) for n_rhs columns (Sec. IV.B product).  x, y: device,
 * column major N x n_rhs, leading dimension ld (complex elements), in the
 * precision's vector type (FP64: complex double; FP32 and BF16X3: complex
 * float).  The block storage precision is p; accumulation is FP32 for FP32
 * and BF16X3, FP64 otherwise.  x and y must not overlap.  FP64 and FP32 take
 * any n_rhs (in passes of four right-hand sides when the handle was built with
 * max_rhs >= 2, else one at a time); BF16X3 takes at most max_rhs.
 * Errors: BAD_HANDLE, INVALID_ARG (BF16X3 with n_rhs > max_rhs, ld < N, null,
 * tier not built), DEVICE. */
h2_status h2_matvec(h2_handle h, h2_op op, h2_precision p, const void* x, void* y, int64_t n_rhs,
                    int64_t ld, void* stream);

/* NONE: plain GMRES.  BLOCKDIAG, MLP: flexible GMRES with z_j = P(v_j) on every
 * Arnoldi vector.  MLP_RESTART: at the start of every cycle, c = P(r) with the
 * attached MLP map and w = Z c (one extra product per cycle) give the step
 * x += alpha c with alpha = w^H r / ||w||^2, the multiple of c that minimises
 * ||b - Z x|| (no step when w = 0); the cycles themselves run with the MLP's base
 * map (none or block diagonal) as right preconditioner.  The network sees true
 * residuals only, the inputs it was trained on. */
typedef enum {
    H2_PRECOND_NONE = 0,
    H2_PRECOND_BLOCKDIAG = 1,
    H2_PRECOND_MLP = 2,
    H2_PRECOND_MLP_RESTART = 3
} h2_precond;

typedef struct {
    int32_t restart;        /* Krylov dimension m per cycle (1..127); 50 */
    int32_t max_matvec;     /* budget of products with Z */
    double tol;             /* relative residual ||b - Z x|| / ||b|| */
    int32_t precision;      /* h2_precision of the inner products (FP64 = plain GMRES) */
    double inner_tol;       /* inner tolerance of refinement when precision != FP64 */
    int32_t max_outer;      /* refinement steps when precision != FP64 */
    int32_t precond;        /* h2_precond: right preconditioner (flexible GMRES when not NONE) */
    int32_t use_x0;         /* 1: x holds the initial guess on entry (resume); 0: x0 = 0 */
} h2_gmres_opts;

typedef struct {
    int32_t converged;
    int32_t iterations;     /* Arnoldi steps over all cycles and refinement steps */
    int32_t matvecs;        /* products with Z (any precision) */
    int32_t restarts;       /* GMRES cycles */
    int32_t outer;          /* refinement steps (0 for FP64) */
    double rel_residual;    /* true ||b - Z x|| / ||b||, FP64 product */
    int32_t corrections;    /* learned restart corrections applied (PRECOND_MLP_RESTART, alpha != 0) */
    int32_t reorth;         /* Arnoldi steps that took a second Gram-Schmidt pass */
} h2_gmres_report;

/* Workspace bytes for h2_gmres_solve with opts o (device memory, caller owned). */
h2_status h2_gmres_workspace(h2_handle h, const h2_gmres_opts* o, size_t* bytes);

/* Solve Z x = b for one right-hand side by restarted GMRES(m) from x0 = 0 (or
 * the given x with use_x0 = 1; restarting from a saved iterate resumes a solve):
 * Arnoldi by classical Gram-Schmidt with a second pass only when the first left
 * less than 1/sqrt(2) of ||w|| (the Daniel-Gragg-Kaufman-Stewart test; the
 * count is rep->reorth), Givens rotations on the Hessenberg matrix, all on the
 * device in FP64; the true residual b - Z x is
 * formed after every cycle and decides convergence.  With precision FP32 or
 * BF16X3 the solve is iterative refinement: r = b - Z x in FP64, an inner
 * GMRES in FP64 arithmetic whose products use the lower-precision blocks,
 * x += d.  With a preconditioner P the method is flexible GMRES with right
 * preconditioning: z_j = P(v_j) is stored, w = Z z_j, and x += sum y_j z_j, so P may
 * change between steps (the MLP is nonlinear).  PRECOND_BLOCKDIAG needs
 * h2_precond_blockdiag, PRECOND_MLP and PRECOND_MLP_RESTART need h2_precond_mlp,
 * both first.
 * b, x: device complex double, length N.  Synchronises the stream.
 * Returns OK, NOT_CONVERGED (x holds the last iterate) or an error. */
h2_status h2_gmres_solve(h2_handle h, const void* b, void* x, const h2_gmres_opts* o,
                         h2_gmres_report* rep, void* work, size_t work_bytes, void* stream);

/* Solve Z x = b by BiCGStab (van der Vorst), the iterative method of the paper's
 * experiments (Sec. V), in FP64 on the device: x0 = 0, shadow residual b,
 * deterministic reductions, two products per step; stops when ||s|| or ||r||
 * reaches tol * ||b|| (or on breakdown) and reports the true FP64 residual
 * b - Z x (rep->restarts = rep->outer = 0).  b, x: device complex double,
 * length N; work: h2_bicgstab_workspace bytes.  Synchronises the stream.
 * Returns OK, NOT_CONVERGED (x holds the last iterate) or an error. */
h2_status h2_bicgstab_workspace(h2_handle h, size_t* bytes);
h2_status h2_bicgstab_solve(h2_handle h, const void* b, void* x, double tol, int32_t max_matvec,
                            h2_gmres_report* rep, void* work, size_t work_bytes, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same solve as h2_bicgstab_solve,
 * same kernels and same results, with its workspace in a device array of the
 * library (h2_bicgstab_static_bytes() = 128 MiB, one copy per device, held
 * until the process ends).  It calls no hipMalloc, hipFree, hipHostMalloc or
 * other allocating routine (both entry points read their per-step scalars into
 * pageable host memory).  Limit: the workspace of
 * h2_bicgstab_workspace must fit in the array (N up to about 1.19 million
 * unknowns); larger N returns INVALID_ARG.  The handle's device must be current
 * (INVALID_ARG otherwise).  Every call on one device shares that device's array:
 * calls that overlap in time on one device (any streams, any handles) race and
 * must not be made; the solve initialises everything it reads.  b, x, tol,
 * max_matvec, rep and the stream as for h2_bicgstab_solve; synchronises it. */
size_t h2_bicgstab_static_bytes(void);
h2_status h2_bicgstab_solve_static(h2_handle h, const void* b, void* x, double tol, int32_t max_matvec,
                                   h2_gmres_report* rep, void* stream);

/* Solve Z x_c = b_c for n_rhs right-hand sides at once (the paper's many
 * right-hand sides, Sec. IV.D): every column runs its own restarted GMRES (FP64
 * Arnoldi with the same selective second Gram-Schmidt pass, per column, Givens,
 * own basis and Hessenberg matrix) in lockstep with the
 * others, so that each product is one multi-column product.  precision FP64:
 * plain restarted GMRES; FP32 / BF16X3: iterative refinement with the outer
 * residual b_c - Z x_c in FP64 and the inner solves (to inner_tol relative to
 * the outer residual) on the lower-precision product; BF16X3 needs the tier and
 * n_rhs <= max_rhs.  precond as for h2_gmres_solve (flexible GMRES per column).
 * b, x: device complex double, column c at b + c * ld, ld >= N; x is the start
 * when use_x0, else overwritten.  reps: host array of n_rhs reports.
 * Synchronises the stream.  Returns OK when every column reached tol,
 * NOT_CONVERGED otherwise (x holds the last iterates), or an error. */
h2_status h2_gmres_batch_workspace(h2_handle h, int64_t n_rhs, int64_t ld, const h2_gmres_opts* o, size_t* bytes);
h2_status h2_gmres_solve_batch(h2_handle h, int64_t n_rhs, const void* b, void* x, int64_t ld, const h2_gmres_opts* o,
                               h2_gmres_report* reps, void* work, size_t work_bytes, void* stream);

typedef struct {
    int64_t n_vox, n_clusters, n_leaves, n_far, n_near, depth;
    int64_t near_elems, coupling_elems, basis_elems, transfer_elems;  /* complex counts */
    int64_t coef_rows;             /* sum of cluster ranks */
    int32_t max_rank, min_leaf_rank;
    int64_t dev_bytes;             /* planned buffer size */
    double bytes_fp64;             /* algorithmic bytes of one FP64 product with 3 columns */
    double flops_fp64;             /* real flops of one product with 3 columns */
    int64_t near_stored_elems;     /* complex entries of the near blocks held on the device
                                      (near_elems unless identical blocks are stored once) */
    int64_t near_unique;           /* distinct near blocks held */
    int64_t near_passes;           /* near-field launches of one full-mode product (1, or several
                                      passes over the distinct blocks when they are stored once) */
    int64_t coupling_owned_elems;  /* coupling entries streamed per product in the symmetric
                                      coupling mode (0: mode not available) */
    int64_t coupling_owned_cols;   /* their columns (one partial of 3 complex each) */
    int64_t near_tiles;            /* tiles of the tiled near field (0: not available) */
    int64_t near_tile_steps;       /* their steps: one stored block each, applied to up to 16
                                      target leaves at once */
} h2_stats_t;

h2_status h2_stats(h2_handle h, h2_stats_t* out);

/*
 * Per-leaf preconditioners.
 *
 * Block diagonal: z_t = (Z_tt)^-1 r_t per leaf t, Z_tt = I + sigma k^2 V G_tt diag(chi_t)
 * on each component; the inverses are formed on the device (Gauss-Jordan with
 * partial pivoting on [Z_tt | I]) into a caller buffer of h2_precond_blockdiag_bytes.
 *
 * Learned: one MLP shared by all leaves (two hidden ReLU layers; bf16 weights,
 * FP32 master weights and accumulation).  A leaf's input is
 * x = [Re r_t / s, Im r_t / s, Re chi_t] (unknowns 3i + c of the leaf's voxels in
 * tree order, zero padded to n_pad voxels: n_in = 7 n_pad), its output
 * y = [Re z_t, Im z_t] / s (n_out = 6 n_pad), s = ||r|| / sqrt(N).
 * Parameter block (device, caller owned, h2_mlp_sizes bytes): FP32 master weights
 * W1 (n_hidden x n_in, row major), b1, W2, b2, W3 (n_out x n_hidden), b3; then the
 * Adam moments m and v; then the bf16 copy used by the passes.
 */
typedef struct { int32_t n_in, n_hidden, n_out; } h2_mlp_dims;

h2_status h2_mlp_sizes(const h2_mlp_dims* dims, int64_t batch, size_t* param_bytes, size_t* work_bytes);
/* Upload master weights (host, float32, the layout above), zero the Adam moments. */
h2_status h2_mlp_set(const h2_mlp_dims* dims, void* params, const float* master_host, void* stream);
h2_status h2_mlp_get(const h2_mlp_dims* dims, const void* params, float* master_host, void* stream);
/* Y (n x n_out) = MLP(X (n x n_in)), device row-major float32. */
h2_status h2_mlp_forward(const h2_mlp_dims* dims, void* params, const float* X, float* Y, int64_t n, void* work,
                         size_t work_bytes, void* stream);
/* Gradients (master layout, device) and loss 0.5/n sum ||Y - T||^2 (device float). */
h2_status h2_mlp_grad(const h2_mlp_dims* dims, void* params, const float* X, const float* T, int64_t n, float* grad,
                      float* loss, void* work, size_t work_bytes, void* stream);
/* Adam (beta 0.9, 0.999, eps 1e-8) over minibatches: epoch e visits rows
 * order[e n .. e n + n) (device int32, caller-drawn permutations) in slices of
 * `batch`; epoch_loss_host (optional, epochs floats) receives mean minibatch losses. */
h2_status h2_mlp_train(const h2_mlp_dims* dims, void* params, const float* X, const float* T, int64_t n,
                       const int* order, int32_t epochs, int32_t batch, float lr, float* epoch_loss_host, void* work,
                       size_t work_bytes, void* stream);

h2_status h2_leaf_count(h2_handle h, int32_t* n_leaves, int32_t* max_leaf);
/* Halo inputs: nbr (host, n_leaves x slots int32, leaves numbered in cluster order,
 * -1 for none) lists each leaf's neighbour leaves; the features then end with
 * 6 values per slot, the neighbour's mean [Re r_c, Im r_c] / s over its voxels
 * (c = 0..2), and n_in = 7 n_pad + 6 slots.  The library keeps a device copy and an
 * n_leaves x 6 buffer of means (so calls on one handle that overlap race).
 * slots = 0 removes the halo.  Detaches any attached MLP. */
h2_status h2_leaf_halo(h2_handle h, const int32_t* nbr, int32_t slots);
/* Features (n_leaves x (7 n_pad + 6 halo slots)) of a residual r (device complex double, length N);
 * leaves in cluster order.  scratch: 64 bytes of device memory. */
h2_status h2_leaf_features(h2_handle h, int32_t n_pad, const void* r, float* X, void* scratch, void* stream);
/* Targets (n_leaves x 6 n_pad) [Re e_t, Im e_t] / s with s from ||r|| (same scaling as the features). */
h2_status h2_leaf_targets(h2_handle h, int32_t n_pad, const void* e, const void* r, float* T, void* scratch,
                          void* stream);
h2_status h2_precond_blockdiag_bytes(h2_handle h, size_t* bytes);
/* Form the leaf inverses into buf; INVALID_ARG if a leaf block is singular. Synchronises.
 * buf (caller memory) is read by every later BLOCKDIAG application and by an MLP
 * attached with that base: keep it alive, unchanged, while the handle uses them. */
h2_status h2_precond_blockdiag(h2_handle h, void* buf, size_t bytes, void* stream);
/* Attach an MLP (parameters stay caller owned) for PRECOND_MLP solves.  base:
 * PRECOND_NONE (z = MLP output) or PRECOND_BLOCKDIAG (z = block-diagonal solve
 * plus the MLP output, a learned correction on top of the fallback; needs
 * h2_precond_blockdiag first). */
h2_status h2_precond_mlp(h2_handle h, const h2_mlp_dims* dims, int32_t n_pad, void* params, int32_t base);
/* z = P(r) once, outside a solve (r, z: distinct device complex double vectors of
 * length N, caller order); work: device memory of h2_precond_apply_bytes (0 for
 * BLOCKDIAG).  Asynchronous on the stream. */
h2_status h2_precond_apply_bytes(h2_handle h, int32_t precond, size_t* bytes);
h2_status h2_precond_apply(h2_handle h, int32_t precond, const void* r, void* z, void* work, size_t work_bytes,
                           void* stream);

/* Kernel families of the product, in launch order. */
enum {
    H2_K_PROLOGUE = 0,      /* U = chi . x, tree permutation */
    H2_K_LEAF_FORWARD = 1,  /* X_t = V_t^T U_t */
    H2_K_UPWARD = 2,        /* X_p = sum T_c^T X_c */
    H2_K_COUPLING = 3,      /* Y_t = sum S_ts X_s */
    H2_K_DOWNWARD = 4,      /* Y_c += T_c Y_p */
    H2_K_NEAR = 5,          /* near field + leaf backward + epilogue; in the symmetric
                               near mode the near field alone (own rows and the partials
                               of the other leaf of each streamed pair) */
    H2_K_NEAR_FINISH = 6,   /* symmetric near mode: partials + leaf backward + epilogue */
    H2_K_COUPLING_RECV = 7, /* symmetric coupling mode: partials S_ts^T X_t added to Y_s */
    H2_K_FAMILIES = 8
};

typedef struct {
    double ms[H2_K_FAMILIES];        /* summed device time per family */
    int64_t launches[H2_K_FAMILIES]; /* launches per family */
} h2_kernel_times;

/* Near-field mode of the FP64 and FP32 single-vector products.  The scalar
 * kernel matrix is symmetric (Sec. II: G depends on |r - r'| only), and when the
 * description's near blocks satisfy G_st = G_ts^T bit for bit (checked at
 * build), the library can stream each unordered leaf pair once: one leaf of the
 * pair adds G_ts u_s to its rows and writes G_ts^T u_t for the other, which adds
 * it when it finishes.  This halves the near-field stream; results agree with
 * the full mode to rounding (the sums are taken in another order).
 *   set: -1 query only, 0 stream every ordered block, 1 the symmetric mode
 *   *mode: the mode in use after the call; *available: 1 if the symmetric mode
 *   can be used (either output may be NULL).
 * Handles start in the symmetric mode when it is available and the near blocks
 * are streamed from memory; when identical blocks are stored once (see
 * H2_BUILD_KEEP_ALL_NEAR) they are read from the caches and handles start in the
 * full mode, which is then the faster one.  The multi-RHS
 * products (n_rhs > 1) and the BF16x3 tier stream every block in both modes.
 * Errors: BAD_HANDLE; INVALID_ARG for set outside {-1, 0, 1} or set = 1 when the
 * mode is not available. */
h2_status h2_near_mode(h2_handle h, int32_t set, int32_t* mode, int32_t* available);

/* Coupling mode of the FP64 and FP32 single-vector products.  G is symmetric and
 * the product uses one basis per cluster for rows and columns, so a description
 * whose couplings satisfy S_st = S_ts^T bit for bit (h2gen's symmetrised
 * couplings; checked at build for every admissible pair, ranks up to 64) lets
 * the library stream each unordered pair once: the owning cluster adds
 * S_ts X_s to its coefficients and writes S_ts^T X_t for the other, which adds
 * those partials before the backward transformation.  This halves the coupling
 * stream; results agree with the full mode to rounding.  Handles start in the
 * full mode: on MI355X the symmetric kernel (transposed products of FP64 rows of
 * rank up to 16 on the matrix cores, a butterfly sum per column otherwise) and the
 * pass that adds the partials take about as long for half the bytes as the full
 * kernel for all of them.
 *   set: -1 query only, 0 every ordered block, 1 the symmetric mode
 *   *mode, *available: as for h2_near_mode (either may be NULL).
 * The multi-RHS products and the BF16x3 tier stream every block.
 * Errors: BAD_HANDLE; INVALID_ARG for set outside {-1, 0, 1} or set = 1 when the
 * mode is not available. */
h2_status h2_coupling_mode(h2_handle h, int32_t set, int32_t* mode, int32_t* available);

/* Tiled near field of the single-vector FP64 and FP32 products in the full near
 * mode, available when identical near blocks are stored once (the default on
 * uniform voxel grids; Sec. IV.B's near-field block products, unchanged).  Leaves
 * consecutive in tree order form tiles of 16; a tile applies each stored block
 * that its leaves use to all of their sources at once, on the matrix cores
 * (16 x 16 x 4 products in the tier's precision; the block is read once per tile
 * instead of once per leaf pair), each complex product as three real ones, Gr Ur,
 * Gi Ui and (Gr + Gi)(Ur + Ui).  Results agree with the per-leaf kernel to
 * rounding (the products are formed and summed in another order).
 *   set: -1 query only, 0 the per-leaf kernel, 1 the tiled kernel
 *   *on: 1 if full-mode FP64 and FP32 products use the tiles after the call;
 *   *available: 1 if the handle has tiles (either output may be NULL).
 * Handles with tiles start with them on.  The symmetric near mode, the BF16x3
 * tier and the multi-RHS products do not use them.
 * Errors: BAD_HANDLE; INVALID_ARG for set outside {-1, 0, 1} or set = 1 without
 * tiles. */
h2_status h2_near_tiles(h2_handle h, int32_t set, int32_t* on, int32_t* available);

/* Diagnostics: with enable = 1, later products on h bracket every kernel
 * family with HIP events on the stream it runs on (the product's stream, or the
 * handle's side stream for the early near-field passes, which keep running
 * beside the couplings: a family can then count two intervals per product);
 * h2_profile_read waits for those events, returns the summed times since the
 * last read, and resets them.  enable = 0 stops recording.  Errors: BAD_HANDLE,
 * INVALID_ARG, DEVICE. */
h2_status h2_profile_enable(h2_handle h, int enable);
h2_status h2_profile_read(h2_handle h, h2_kernel_times* out);

/*
 * Batched BF16x3 tier (representations built with tier bit 1 << H2_BF16X3).
 *
 * Every block product of the H^2 product becomes a complex block GEMM over
 * W = 3 * n_rhs columns (the paper's H^2 x dense product for many right-hand
 * sides, Sec. IV.D), done in real arithmetic on the matrix cores with each
 * operand split into bf16 hi + lo parts (hi*hi + hi*lo + lo*hi, FP32
 * accumulation).  Vectors are complex float (complex64), column major, ld >= N.
 * h2_matvec with p = H2_BF16X3 runs one representation this way.
 *
 * A group runs several representations (geometries of any size, each with its
 * own n_rhs) phase by phase in shared launches: leaf forward, upward levels
 * (aligned from the leaves), couplings, downward levels (aligned from the top),
 * near field; the launch sequence is captured in a HIP graph on first use for
 * a given set of vector pointers, column counts and op, and replayed after.
 * Members must outlive the group; the group buffer is caller-owned device
 * memory of at least h2_group_plan bytes.
 */
typedef struct h2_group_s* h2_group;

h2_status h2_group_plan(const h2_handle* members, int32_t n, size_t* dev_bytes);
h2_status h2_group_build(const h2_handle* members, int32_t n, void* dev_buffer, size_t dev_bytes,
                         void* stream, h2_group* out);
/* y[i] = op(x[i]) for every member i (n_rhs[i] = 0 skips a member).  Stream ordered. */
h2_status h2_group_matvec(h2_group g, h2_op op, const void* const* x, void* const* y, const int64_t* n_rhs,
                          const int64_t* ld, void* stream);
/* Autotuner: times the column tile widths 32, 64 and 128 of the block GEMM on the
 * given vectors, phase by phase, and keeps each phase's fastest (*tile receives the
 * near-field phase's).  Synchronises. */
h2_status h2_group_tune(h2_group g, h2_op op, const void* const* x, void* const* y, const int64_t* n_rhs,
                        const int64_t* ld, void* stream, int32_t* tile);
/* Set the column tile of every phase (32, 64, 128; 0 keeps the tiles) and graph use (0 / 1). */
h2_status h2_group_set(h2_group g, int32_t tile, int32_t use_graph);
void h2_group_destroy(h2_group g);

/* Release the handle's host metadata.  Never frees caller memory.  NULL is ignored. */
void h2_destroy(h2_handle h);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* h2_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* H2VIE_H */
