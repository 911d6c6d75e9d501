// Deterministic wave64/block reductions.
#pragma once

#include <hip/hip_runtime.h>

namespace fo {

// reductions: wave64 DPP, then LDS across the waves of a block

// x of the lane that the DPP control CTRL selects, 0 where it selects none
// or the row/bank mask disables the lane (register-only cross-lane read).
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ double dpp_read(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROW_MASK, BANK_MASK, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROW_MASK, BANK_MASK, true);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave (all lanes active), valid in every lane:
// prefix sums within each row of 16 lanes (row_shr 1, 2, 3, then 4 and 8 on
// the upper banks), the row totals chained by row_bcast 15 and 31 into lane
// 63, then read from lane 63.  A fixed order: the same inputs give the same
// bits in every wave.
__device__ __forceinline__ double wave_sum(double x)
{
    double v = x + dpp_read<0x111, 0xf, 0xf>(x);
    v += dpp_read<0x112, 0xf, 0xf>(x);
    v += dpp_read<0x113, 0xf, 0xf>(x);
    v += dpp_read<0x114, 0xf, 0xe>(v);
    v += dpp_read<0x118, 0xf, 0xc>(v);
    v += dpp_read<0x142, 0xa, 0xf>(v);
    v += dpp_read<0x143, 0xc, 0xf>(v);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// x of lane (lane ^ 1) or (lane ^ 2) within each group of four (DPP quad_perm).
template <int XOR, typename T>
__device__ __forceinline__ T quad_xor(T x)
{
    static_assert(XOR == 1 || XOR == 2, "quad lanes");
    constexpr int QP = XOR == 1 ? 0xB1 : 0x4E;  // (1,0,3,2) or (2,3,0,1)
    if constexpr (sizeof(T) == 4) {
        return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), QP, 0xf, 0xf, false));
    } else {
        const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), QP, 0xf, 0xf, false);
        const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), QP, 0xf, 0xf, false);
        return __hiloint2double(hi, lo);
    }
}

// Sum over a 256-thread block; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds /*[4]*/)
{
    v = wave_sum(v);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = (lds[0] + lds[1]) + (lds[2] + lds[3]);
    __syncthreads();
    return s;
}

// Deterministic sum of n partials by one 256-thread block (thread 0 gets it).
__device__ __forceinline__ double block_sum_partials(const double *part, int n, double *lds)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
    return block_sum(s, lds);
}

// Sum over a block of any size that is a multiple of 64 (at most 1024
// threads): wave sums, then wave 0 sums the wave totals (a fixed order).
// Valid in every lane of wave 0.
__device__ __forceinline__ double block_sum_any(double v, double *lds /*[16]*/)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x < 64) s = wave_sum(lane < nw ? lds[lane] : 0.0);
    __syncthreads();
    return s;
}

// block_sum_any for the last use of lds in a kernel (no trailing barrier).
__device__ __forceinline__ double block_sum_last(double v, double *lds /*[16]*/)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    return threadIdx.x < 64 ? wave_sum(lane < nw ? lds[lane] : 0.0) : 0.0;
}

// Two block sums in one pass (lds[32]); valid in every lane of wave 0.
__device__ __forceinline__ void block_sum2_any(double &a, double &b, double *lds /*[32]*/)
{
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    if (lane == 0) {
        lds[w] = a;
        lds[16 + w] = b;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        a = wave_sum(lane < nw ? lds[lane] : 0.0);
        b = wave_sum(lane < nw ? lds[16 + lane] : 0.0);
    }
    __syncthreads();
}

// Every thread of the block gets the same fixed-order sum of n partials.
__device__ __forceinline__ double block_sum_partials_any(const double *part, int n, double *lds)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
    s = block_sum_any(s, lds);
    if (threadIdx.x == 0) lds[0] = s;
    __syncthreads();
    s = lds[0];
    __syncthreads();
    return s;
}

// Sum of n partials by the first wave of a block, in a fixed order (lane
// strided sums, then a butterfly): every block that calls it gets the same
// value.  Valid in all lanes of wave 0.
__device__ __forceinline__ double wave0_sum_partials(const double *part, int n)
{
    double s = 0.0;
    for (int i = (int)(threadIdx.x & 63); i < n; i += 64) s += part[i];
    return wave_sum(s);
}

// Partial sums read in two steps, so that the loads overlap other work:
// part_issue() loads the first KP strides of partials into registers
// (indices clamped to n - 1: no branch, every load in bounds, n >= 1) and
// part_finish() drops the clamped copies, adds the partials beyond KP
// strides and returns the thread's strided sum.  The order of the additions
// is that of the plain strided loop (s = 0; s += part[i], i = lane, lane +
// width, ...), so the reductions built on it keep their results bit for bit.
template <int KP>
struct PartLoad {
    double v[KP];
};

template <int KP>
__device__ __forceinline__ void part_issue(PartLoad<KP> &pl, const double *__restrict__ part, int n,
                                           int lane, int width)
{
#pragma unroll
    for (int k = 0; k < KP; ++k) pl.v[k] = part[min(lane + k * width, n - 1)];
}

template <int KP>
__device__ __forceinline__ double part_finish(const PartLoad<KP> &pl, const double *__restrict__ part,
                                              int n, int lane, int width)
{
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < KP; ++k)
        if (lane + k * width < n) s += pl.v[k];
    for (int i = lane + KP * width; i < n; i += width) s += part[i];
    return s;
}

}  // namespace fo
