// Host-side state of a warm-start model (shared by the model entry points
// and the warm plans).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/rpod.h"

struct rpod_warm_s {
    rpod_warm_desc d;
    rpod_warm_layout L;
    char* ws = nullptr;
    hipStream_t st = nullptr;
    int64_t mP = 0;        // rows of the bank (roundup(m, 256))
    int Kr = 0;            // 8 r
    int bank_cols = 0;     // roundup(Kr, 128): zero columns after the bases
    int64_t nPb = 0;       // roundup(Kr, 256): rows of bank^T products
    int nsplit = 0;        // row splits of bank^T products
    int64_t split_rows = 0;
    int rpad = 0;          // roundup(r, 16)
    // scratch offsets (bytes)
    size_t o_H1 = 0, o_H2 = 0, o_dA1 = 0, o_dA2 = 0, o_C = 0, o_dZ = 0, o_lossn = 0, o_loss = 0;
    size_t o_stage = 0, o_Zp = 0, o_Zt = 0, o_args = 0, args_bytes = 0;
    int64_t adam_t = 0;    // Adam steps taken
    template <typename T>
    T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};
