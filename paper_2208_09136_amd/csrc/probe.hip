// probe.hip -- VALU issue-rate probe of the GPU the library runs on.
//
// The line sweeps and counting passes are bound by vector-ALU issue and LDS,
// not by HBM, so their roofline is the chip's VALU rate.  This probe measures
// that rate per instruction class: every lane runs PROBE_CHAINS independent
// dependency chains of one instruction, many waves per SIMD hide the chain
// latency, and the rate is the executed lane-operations over the kernel time.
// The instruction is written in inline assembly (register operands only, no
// memory access) so that the compiler can neither fold the chains nor pick
// another encoding; the chains' end values are stored so that nothing is dead.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace rqa {

constexpr int PROBE_CHAINS = 16;
constexpr int PROBE_UNROLL = 8;
constexpr int PROBE_BLOCK = 256;

// KIND 0: v_add_f32 (32-bit float add), KIND 1: v_add_u32 (32-bit integer
// add), KIND 2: v_max_u32 (32-bit integer max), KIND 3: v_add_u32 with a
// scalar-register operand (which drops the add to the rate of KIND 2).
template <int KIND>
__device__ __forceinline__ void probe_op(uint32_t& x, uint32_t y, uint32_t ys)
{
    if constexpr (KIND == 0) asm volatile("v_add_f32 %0, %1, %0" : "+v"(x) : "v"(y));
    else if constexpr (KIND == 1) asm volatile("v_add_u32 %0, %1, %0" : "+v"(x) : "v"(y));
    else if constexpr (KIND == 2) asm volatile("v_max_u32 %0, %1, %0" : "+v"(x) : "v"(y));
    else asm volatile("v_add_u32 %0, %1, %0" : "+v"(x) : "s"(ys));
}

template <int KIND>
__global__ void __launch_bounds__(PROBE_BLOCK) k_valu_probe(uint32_t* __restrict__ out, uint32_t iters, uint32_t seed)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t x[PROBE_CHAINS];
    const uint32_t y = seed ^ tid;
    const uint32_t ys = seed;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) x[c] = tid * 2654435761u + (uint32_t)c;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u) {
#pragma unroll
            for (int c = 0; c < PROBE_CHAINS; ++c) probe_op<KIND>(x[c], y, ys);
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) acc ^= x[c];
    out[tid] = acc;
}

uint64_t valu_probe_threads(uint32_t blocks) { return (uint64_t)blocks * PROBE_BLOCK; }

// Lane-operations of one launch: threads x iterations x unroll x chains.
double valu_probe_lane_ops(uint32_t blocks, uint32_t iters)
{
    return (double)blocks * PROBE_BLOCK * (double)iters * PROBE_UNROLL * PROBE_CHAINS;
}

hipError_t launch_valu_probe(hipStream_t st, int kind, uint32_t blocks, uint32_t iters, uint32_t* out)
{
    switch (kind) {
    case 0: hipLaunchKernelGGL(k_valu_probe<0>, dim3(blocks), dim3(PROBE_BLOCK), 0, st, out, iters, 0x9E3779B9u); break;
    case 1: hipLaunchKernelGGL(k_valu_probe<1>, dim3(blocks), dim3(PROBE_BLOCK), 0, st, out, iters, 0x9E3779B9u); break;
    case 2: hipLaunchKernelGGL(k_valu_probe<2>, dim3(blocks), dim3(PROBE_BLOCK), 0, st, out, iters, 0x9E3779B9u); break;
    default: hipLaunchKernelGGL(k_valu_probe<3>, dim3(blocks), dim3(PROBE_BLOCK), 0, st, out, iters, 0x9E3779B9u); break;
    }
    return hipGetLastError();
}

}  // namespace rqa
