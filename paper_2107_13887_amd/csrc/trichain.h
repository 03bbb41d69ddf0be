// Chained 64-row block triangular solves, shared by the dense weight solve and the greedy's level
// close: one launch, a 64-lane workgroup (one wave) per block, finished blocks published to later
// ones through done flags. Tickets follow the order in which workgroups start, so a workgroup only
// waits for blocks owned by workgroups already running, whatever the grid size. A wait polls a
// bounded number of times and then raises a fault flag instead of hanging; every other wait that
// sees the flag ends too.
#pragma once

#include <hip/hip_runtime.h>

namespace rbf {

constexpr int TC_NB = 64;
// Default bound on the polls of one wait (each after a short sleep, seconds in all): far beyond
// any chain, it only ends a wait that could never be met.
constexpr unsigned long long TC_SPIN_LIMIT = 1ull << 22;

// Dv = inv(L) for the lower-triangular 64 x 64 block L in LDS (rows and columns past the matrix
// are identity): lane t forms column t by forward substitution (x_j = r_j / L_jj with the
// reciprocal formed beforehand, then r_i -= L_ij x_j for i > j), the column of L read as
// broadcasts. The workgroup is the single wave; rl is LDS scratch of 64.
__device__ __forceinline__ void tc_tri_inverse(const double (*L)[TC_NB + 1], double (*Dv)[TC_NB + 1], double *rl)
{
    const int t = threadIdx.x;
    rl[t] = 1.0 / L[t][t];
    __syncthreads();
    double r[TC_NB];
#pragma unroll
    for (int i = 0; i < TC_NB; ++i) r[i] = i == t ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < TC_NB; ++j) {
        const double xj = r[j] * rl[j];
        r[j] = xj;
#pragma unroll
        for (int i = j + 1; i < TC_NB; ++i) r[i] = __builtin_fma(-L[i][j], xj, r[i]);
    }
#pragma unroll
    for (int j = 0; j < TC_NB; ++j) Dv[j][t] = r[j];
}

// Workgroup-uniform wait until *flag reaches want (relaxed polls, then one acquire); false when
// the wait gave up or another wait already did (*fault raised).
__device__ __forceinline__ bool tc_wait(const int32_t *flag, int32_t want, int32_t *fault,
                                        unsigned long long limit, int32_t &ok_sh)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long spins = 0;
        int32_t ok = 1;
        while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
            if (spins++ >= limit ||
                ((spins & 63) == 0 && __hip_atomic_load(fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (!ok) __hip_atomic_store(fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        ok_sh = ok;
    }
    __syncthreads();
    return ok_sh != 0;
}

// Publish the workgroup's block: its stores, then a release store of the done flag.
__device__ __forceinline__ void tc_publish(int32_t *flag)
{
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace rbf
