// Kernel-sum launch interface shared by the kernels (ksum.hip) and the host planner that sizes
// and orders their launches (ksum_host.cpp). Internal: not part of the C ABI.
#pragma once

#include "internal.h"

namespace rbf {
namespace ksum {

constexpr int BLOCK = 256;
constexpr int TILE = 256;
constexpr int CHUNK = 4;                  // points per lane in the compaction
constexpr int CBLK = BLOCK * CHUNK;       // points per compaction block

struct KArgs {
    int32_t n_levels;
    int32_t n_split;
    SumLevel lv[RBF_MAX_LEVELS];
    const double *xc;               // [DIM][ld_ctrl]
    const double *alpha;            // [DIM][ld_ctrl]
    int64_t ld_ctrl;
    const int32_t *work;            // reduced point list, or null for the identity
    const int32_t *out_perm;        // resident geometry: output index of stored point w (-1: padding)
    const int64_t *n_work_dev;      // device-side count (null: use n_work)
    int64_t n_work;
    const double *xp;
    int64_t ld_p;
    const double *dwall;
    const double *base;
    double sign;
    double *out;
    int64_t ld_out;
    double *partial;                // [n_split][DIM][ld_part]
    int64_t ld_part;
    unsigned long long *pairs;      // evaluated (point, control) pairs are added here, or null
    int64_t n_live;                 // rows from here on need no level (-1: every row may)
    const double *block_box;        // resident geometry: box of every BOXROWS stored rows [n / BOXROWS][2 DIM], or null
    const int32_t *order;           // resident geometry: row group of workgroup x (a permutation), or null: group x
};

// Enqueue the kernel-sum grid (one workgroup per BLOCK * P rows, gridDim.y splits of the control
// lists) for the given dimension, points per lane, FP32 pair form and basis. start / stop, when
// given, receive the kernel's own start and end times (hipExtLaunchKernel), which leave out the
// host's launch latency that events recorded around the launch on an idle stream would include.
void launch_sum(const KArgs &a, dim3 grid, int dim, int P, bool mixed, int32_t basis, hipStream_t s,
                hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// Sum the split partials in split order and write the final values.
void launch_finalize(const KArgs &a, int dim, int blocks, hipStream_t s);
// Stable compaction of {v : d_v < dmax} into work[0, *n_work), +0.0 written to every dropped
// point's dim components of out; counts needs one int per CBLK points.
void launch_reduce(const double *d, int64_t n, double dmax, int32_t *counts, int64_t *n_work,
                   int32_t *work, double *out, int32_t dim, hipStream_t s);

}  // namespace ksum
}  // namespace rbf
