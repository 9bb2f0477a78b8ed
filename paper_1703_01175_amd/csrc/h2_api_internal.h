// Declarations shared by the host translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/h2vie.h"
#include "h2_internal.h"
#include "h2_batch.h"

#include <vector>

namespace h2 {

// Per-handle device scratch beyond the product's U / X / Y arrays (bytes).
inline size_t aux_scratch_bytes(int64_t n_vox, int coef_rows) {
    (void)coef_rows;
    return size_t(n_vox) * kNcomp * 8 * 2 + 4096;   // two complex-float vectors + flags
}

// Element conversions (h2_convert.hip).
hipError_t launch_convert_fp32(const double2* src, float2* dst, int64_t n, hipStream_t s);
hipError_t launch_split_bf16(const double2* src, uint32_t* hi, uint32_t* lo, int64_t n, hipStream_t s);
hipError_t launch_vec_to_fp32(const double2* src, float2* dst, int64_t n, hipStream_t s);
hipError_t launch_vec_to_fp64(const float2* src, double2* dst, int64_t n, hipStream_t s);

// Preconditioner applications (h2_learn.hip).
hipError_t launch_bd_apply(const LeafInfo& li, const int* perm, const double2* inv, const double2* r, double2* z,
                           hipStream_t s);
// MLP correction z = MLP(r) per leaf; X, H1, H2, Y: activations of n_leaves rows; norm: 1 double
hipError_t mlp_apply_handle(h2_handle h, const double2* r, double2* z, float* X, float* H1, float* H2, float* Y,
                            double* norm, hipStream_t s);
size_t mlp_apply_work_bytes(h2_handle h);

// Handle accessors (h2vie_api.cpp) for the solver translation unit.
const DevH2* handle_dev(h2_handle h);
const LevelLaunch* handle_levels(h2_handle h);
void* handle_aux(h2_handle h, size_t* bytes);
bool handle_live(h2_handle h);
h2_status handle_fail(h2_status st, const char* msg);

// Batched BF16x3 tier (h2_batch_api.cpp)
// near_off / coup_off: offset of each near / far pair's block in the FP64 arrays as held
// on the device (coup_off null: the description's offsets)
h2_status plan_batch(const h2_host_desc* d, int max_rhs, const int64_t* near_off, const int64_t* coup_off,
                     BatchHost& B);
size_t group_need(const h2_handle* hs, int n);
size_t group_need_batch(BatchHost* B);
h2_status group_create(const h2_handle* hs, int n, void* mem, size_t bytes, hipStream_t s, h2_group* out);
h2_status group_run(h2_group g, int op, const void* const* x, void* const* y, const int64_t* n_rhs,
                    const int64_t* ld, hipStream_t s);
void group_destroy(h2_group g);
h2_status group_autotile(h2_group g, const void* x, void* y, int64_t n_rhs, int64_t ld, hipStream_t s);

// Event pairs around kernel families; read back (and summed) on demand.
struct EventProfiler : Profiler {
    struct Rec { int family; hipEvent_t a, b; };
    std::vector<Rec> open, done;
    std::vector<hipEvent_t> pool;
    hipEvent_t take() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void begin(int family, hipStream_t s) override {
        hipEvent_t a = take();
        if (!a) return;
        (void)hipEventRecord(a, s);
        open.push_back({family, a, nullptr});
    }
    void end(int family, hipStream_t s) override {
        for (size_t i = open.size(); i-- > 0;)
            if (open[i].family == family && open[i].b == nullptr) {
                hipEvent_t b = take();
                if (!b) return;
                (void)hipEventRecord(b, s);
                open[i].b = b;
                done.push_back(open[i]);
                open.erase(open.begin() + i);
                return;
            }
    }
    ~EventProfiler() override {
        for (auto& r : done) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        for (auto& r : open) (void)hipEventDestroy(r.a);
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};


constexpr uint32_t kHandleMagic = 0x48325649u;  // "H2VI"

}  // namespace h2

struct h2_handle_s {
    uint32_t magic = h2::kHandleMagic;
    h2::DevH2 dev;
    h2::LevelLaunch lv;
    h2_stats_t stats{};
    char* base = nullptr;
    size_t bytes = 0;
    int device = -1;                    // device current at build (where base lives)
    void* aux = nullptr;
    size_t aux_bytes = 0;
    int tiers = 1;
    h2::EventProfiler* prof = nullptr;
    h2::BatchHost* batch = nullptr;     // BF16x3 batched tier (tier bit 2)
    h2_group self_group = nullptr;      // the handle alone, for h2_matvec with BF16X3
    // preconditioners
    void* bd_buf = nullptr;             // [M_t | I] after elimination, per leaf (caller memory)
    bool bd_ready = false;
    void* mlp_params = nullptr;         // MLP parameter block (caller memory)
    h2_mlp_dims mlp_dims{0, 0, 0};
    int mlp_npad = 0;
    int mlp_base = 0;                   // H2_PRECOND_NONE, or BLOCKDIAG: z = BD(r) + MLP correction
    int* halo_nbr = nullptr;            // n_leaves x halo_slots neighbour leaves (-1: none), library memory
    float* halo_means = nullptr;        // n_leaves x 6 scaled leaf means of the current input, library memory
    int halo_slots = 0;
    ~h2_handle_s() {
        if (dev.near_side) (void)hipStreamDestroy(dev.near_side);
        if (dev.near_fork) (void)hipEventDestroy(dev.near_fork);
        if (dev.near_join) (void)hipEventDestroy(dev.near_join);
        if (halo_nbr) (void)hipFree(halo_nbr);
        if (halo_means) (void)hipFree(halo_means);
        if (self_group) h2::group_destroy(self_group);
        delete batch;
        delete prof;
    }
};
