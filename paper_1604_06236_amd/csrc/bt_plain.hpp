// Unfused comparison path and the tap-gradient row reduction (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bt_dft.hpp"

namespace bt {

enum PlainInOp : int { IN_NONE = 0, IN_MUL_TAP = 1, IN_DIV_NTAP = 2 };
enum PlainOutOp : int { OUT_NONE = 0, OUT_MUL_TAP = 1, OUT_DIV_NTAP = 2 };
enum PlainTgOp : int { TG_NONE = 0, TG_OUT = 1 };

struct PlainArgs {
    int K, M;
    int64_t nblocks;
    int64_t tap_stride;
    const float *taps;
    const c32 *roots;     // e^{+j 2 pi k / N}, k < N
    const c32 *aux;       // S for the tap term of the adjoint
    c32 *out;
    int *status;
    int conj_io, in_op, out_op, tg_op;
};

// runs all stages; ws0 and ws1 each hold nblocks*N complex values; tg_part
// receives per-block tap-gradient rows when tg_op is set
hipError_t plain_run(const PlainArgs &a, const c32 *in, c32 *ws0, c32 *ws1, float *tg_part,
                     hipStream_t s);

// rows per first-stage chunk of rows_reduce, and the number of chunks (the chunk sums
// go to the scratch rows when there are two or more)
constexpr int64_t ROWS_REDUCE_CHUNK = 16;
inline int64_t rows_reduce_chunks(int64_t rows) { return (rows + ROWS_REDUCE_CHUNK - 1) / ROWS_REDUCE_CHUNK; }

// out[k] = sum_{r < rows} part[r*n + k], fixed order; `scratch` holds
// rows_reduce_chunks(rows)*n floats
hipError_t rows_reduce(const float *part, int64_t rows, int64_t n, float *scratch, float *out,
                       hipStream_t s);

} // namespace bt
