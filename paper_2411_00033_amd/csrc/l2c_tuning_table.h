// l2c_tuning_table.h -- leaf size and rank per size bucket of a ragged batch
// (leg2cheb_batch_plan with tuning = NULL), per precision form.
//
// Written by paper_2411_00033_amd/autotune.py from timings of the ragged batch on an
// MI355X; regenerate it with that script.  Each row covers the lengths n with
// n_max(previous row) < n <= n_max; the last row covers every larger n.  Every row met its
// form's error bound against the FP64 path at rank 24 on the bucket's transforms (FP64:
// E_inf <= 1e-13); the batched forms keep rank <= 16 and leaf <= 64.
// Made 2026-12-03 13:07 UTC.
#pragma once
#include <stdint.h>

namespace l2c {

struct TuneRow {
    int64_t n_max;
    int32_t leaf_size, rank;
};

static const TuneRow kTuneFP64[] = {{512, 32, 18},
                                      {2048, 48, 20},
                                      {8192, 48, 16},
                                      {INT64_MAX, 64, 16}};
static const TuneRow kTuneBatched[] = {{512, 64, 16},
                                      {2048, 32, 16},
                                      {131072, 64, 12},
                                      {INT64_MAX, 64, 16}};

inline int builtin_tuning(int precision, const TuneRow **rows)
{
    if (precision == 0) {
        *rows = kTuneFP64;
        return (int)(sizeof(kTuneFP64) / sizeof(kTuneFP64[0]));
    }
    *rows = kTuneBatched;
    return (int)(sizeof(kTuneBatched) / sizeof(kTuneBatched[0]));
}

}  // namespace l2c
