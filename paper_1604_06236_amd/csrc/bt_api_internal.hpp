// Declarations shared by the C-ABI translation units (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

namespace bt {

extern thread_local std::string g_last_error;
void set_error(const char *what, hipError_t e);
bool supported_km(int K, int M);

// schedule option bit (beside the uniform kernel's options): the entry runs the half-block
// exchange kernel of bt_fused_half.hip in the directions without a tap gradient
constexpr int OPT_HALF_LDS = 32;

// split-precision MFMA path
int split_supported(int K, int M, int compute);
size_t split_workspace_size(int64_t nblocks, int K, int M, int64_t tap_stride, int compute,
                            int with_tapbar);
int split_prepare(int K, int M, int compute);
// direction 0: forward, 1: adjoint (coefficient part)
int split_run(int direction, const void *in, const float *taps, void *out, int64_t nblocks, int K,
              int M, int64_t tap_stride, int compute, void *ws, size_t ws_bytes, void *stream);

} // namespace bt
