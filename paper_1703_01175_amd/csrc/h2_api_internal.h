// Declarations shared by the host translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/h2vie.h"
#include "h2_internal.h"

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

// Handle accessors (h2vie_api.cpp) for the solver translation unit.
const DevH2* handle_dev(h2_handle h);
const LevelLaunch* handle_levels(h2_handle h);
void* handle_aux(h2_handle h, size_t* bytes);
bool handle_live(h2_handle h);
h2_status handle_fail(h2_status st, const char* msg);

}  // namespace h2
