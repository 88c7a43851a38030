// Measurement probes: what a launch of a given size can reach on this GPU.
//
// These kernels compute nothing the library returns.  They bound the tile
// kernels from below: an empty launch (the fixed cost of dispatch and
// completion) and plain reads of a buffer in several shapes (workgroups,
// threads per workgroup, 16-byte loads in flight per lane, loads into
// registers or straight into LDS, arguments in SGPRs at wave start or loaded
// from the kernel-argument segment).  The fastest read of the tile kernel's
// byte count is the floor its launch is compared with.
//
// This file is compiled on its own with kernel-argument preloading enabled:
// kernels whose leading arguments are scalars start with those arguments
// already in SGPRs; a kernel that takes one struct by value loads it from
// memory as every kernel of the library does.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "iqa.h"

namespace iqa_probe {

constexpr int kWave = 64;

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void glb_void;

__device__ __forceinline__ f4v ntload(const float4 *p) {
    return __builtin_nontemporal_load(reinterpret_cast<const f4v *>(p));
}

__device__ __forceinline__ float hsum(f4v v) { return (v.x + v.y) + (v.z + v.w); }

// One float per workgroup, so that no load can be dropped: the wave sums go
// through LDS, in a fixed order.
__device__ __forceinline__ void block_out(float acc, float *out) {
    for (int st = 32; st > 0; st >>= 1) acc += __shfl_xor(acc, st, kWave);
    __shared__ float part[16];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    if (lane == 0) part[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) s += part[w];
        out[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(1024) void probe_empty() {}

// Contiguous chunk of `per_block` float4s per workgroup; each lane keeps
// LOADS loads in flight (stride: the workgroup's width), then adds them.
template <int LOADS>
__device__ __forceinline__ void read_regs_body(const float4 *src, int64_t n4, int64_t per_block,
                                               int32_t width, float *out) {
    const int64_t b0 = (int64_t)blockIdx.x * per_block;
    const int64_t b1 = b0 + per_block < n4 ? b0 + per_block : n4;
    const int64_t w = width;   // blockDim.x, passed in so that no load precedes the first read
    float acc = 0.f;
    int64_t i = b0 + threadIdx.x;
    for (; i + (LOADS - 1) * w < b1; i += LOADS * w) {
        f4v v[LOADS];
#pragma unroll
        for (int u = 0; u < LOADS; ++u) v[u] = ntload(src + i + u * w);
#pragma unroll
        for (int u = 0; u < LOADS; ++u) acc += hsum(v[u]);
    }
    for (; i < b1; i += w) acc += hsum(ntload(src + i));
    block_out(acc, out);
}

// Arguments as scalars: preloaded into SGPRs at wave start.
template <int LOADS>
__global__ __launch_bounds__(1024) void probe_read_regs(const float4 *src, int64_t n4,
                                                        int64_t per_block, int32_t width,
                                                        float *out) {
    read_regs_body<LOADS>(src, n4, per_block, width, out);
}

// The same read with its arguments in one struct, loaded from memory.
struct ReadArgs {
    const float4 *src;
    int64_t n4;
    int64_t per_block;
    int32_t width;
    float *out;
};

template <int LOADS>
__global__ __launch_bounds__(1024) void probe_read_regs_struct(ReadArgs a) {
    read_regs_body<LOADS>(a.src, a.n4, a.per_block, a.width, a.out);
}

// Loads straight into LDS (gfx950 global_load_lds_dwordx4: each lane's 16
// bytes land at the wave's LDS base + 16 * lane, no VGPRs held), LOADS per
// lane in flight, then each lane adds back its own slots.  Dynamic LDS:
// LOADS KiB per wave.
template <int LOADS>
__global__ __launch_bounds__(1024) void probe_read_lds(const float4 *src, int64_t n4,
                                                       int64_t per_block, int32_t width,
                                                       float *out) {
    extern __shared__ float4 slots[];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    float4 *mine = slots + (int64_t)wave * LOADS * kWave;
    const int64_t b0 = (int64_t)blockIdx.x * per_block;
    const int64_t b1 = b0 + per_block < n4 ? b0 + per_block : n4;
    const int64_t w = width;
    float acc = 0.f;
    int64_t i = b0 + threadIdx.x;
    for (; i + (LOADS - 1) * w < b1; i += LOADS * w) {
#pragma unroll
        for (int u = 0; u < LOADS; ++u)
            __builtin_amdgcn_global_load_lds((glb_void *)(src + i + u * w),
                                             (lds_void *)(mine + u * kWave), 16, 0, 0);
        __builtin_amdgcn_s_waitcnt(0);   // the wave's LDS writes have landed
#pragma unroll
        for (int u = 0; u < LOADS; ++u) {
            const float4 v = mine[u * kWave + lane];
            acc += (v.x + v.y) + (v.z + v.w);
        }
        __builtin_amdgcn_s_waitcnt(0);   // slots read before the next loads overwrite them
    }
    for (; i < b1; i += w) acc += hsum(ntload(src + i));
    block_out(acc, out);
}

// The register read with wall-clock stamps, in the record layout of the tile
// kernel's timelines (8 uint64 per workgroup at tl[8 * blockIdx.x], from wave
// 0): entry, its first batch of loads summed, its last loads summed, its exit
// once the workgroup's sum is stored, XCC_ID, HW_ID, the workgroup index, and
// 1 << 32 (the word an unsplit tile workgroup writes).
// A stamp is read only after the value it follows is in a register (the
// empty volatile asm needs it), so it cannot move above the loads.
__device__ __forceinline__ uint64_t stamp_after(float v) {
    asm volatile("" ::"v"(v));
    return wall_clock64();
}

template <int LOADS>
__global__ __launch_bounds__(1024) void probe_read_regs_tl(const float4 *src, int64_t n4,
                                                           int64_t per_block, int32_t width,
                                                           float *out, uint64_t *tl) {
    const uint64_t t_entry = wall_clock64();
    const int64_t b0 = (int64_t)blockIdx.x * per_block;
    const int64_t b1 = b0 + per_block < n4 ? b0 + per_block : n4;
    const int64_t w = width;
    float acc = 0.f;
    uint64_t t_first = 0;
    int64_t i = b0 + threadIdx.x;
    for (; i + (LOADS - 1) * w < b1; i += LOADS * w) {
        f4v v[LOADS];
#pragma unroll
        for (int u = 0; u < LOADS; ++u) v[u] = ntload(src + i + u * w);
#pragma unroll
        for (int u = 0; u < LOADS; ++u) acc += hsum(v[u]);
        if (t_first == 0) t_first = stamp_after(acc);
    }
    for (; i < b1; i += w) acc += hsum(ntload(src + i));
    const uint64_t t_last = stamp_after(acc);
    block_out(acc, out);
    if (threadIdx.x < kWave) {
        __builtin_amdgcn_s_waitcnt(0);   // the workgroup's store has landed
        const uint64_t t_end = wall_clock64();
        if (threadIdx.x == 0) {
            uint64_t *r = tl + (int64_t)blockIdx.x * 8;
            r[0] = t_entry;
            r[1] = t_first ? t_first : t_last;
            r[2] = t_last;
            r[3] = t_end;
            r[4] = (uint64_t)__builtin_amdgcn_s_getreg((31 << 11) | 20);   // XCC_ID
            r[5] = (uint64_t)__builtin_amdgcn_s_getreg((31 << 11) | 4);    // HW_ID
            r[6] = (uint64_t)blockIdx.x;
            r[7] = (uint64_t)1 << 32;   // finished its own work, as an unsplit tile workgroup
        }
    }
}

thread_local int g_last_error = 0;

iqa_status status(hipError_t e) {
    if (e == hipSuccess) return IQA_OK;
    g_last_error = (int)e;
    return IQA_ERR_HIP;
}

template <typename... P>
hipError_t launch(void (*fn)(P...), unsigned grid, unsigned block, size_t lds, hipStream_t s,
                  P... args) {
    void *argv[] = {static_cast<void *>(&args)...};
    return hipLaunchKernel(reinterpret_cast<const void *>(fn), dim3(grid), dim3(block), argv, lds,
                           s);
}

template <int L>
iqa_status read_with(int mode, const float4 *src, int64_t n4, int64_t per, float *out,
                     unsigned blocks, unsigned threads, hipStream_t s) {
    switch (mode) {
        case IQA_PROBE_READ_REGS:
            return status(launch(&probe_read_regs<L>, blocks, threads, 0, s, src, n4, per,
                                 (int32_t)threads, out));
        case IQA_PROBE_READ_REGS_STRUCT: {
            ReadArgs a{src, n4, per, (int32_t)threads, out};
            return status(launch(&probe_read_regs_struct<L>, blocks, threads, 0, s, a));
        }
        case IQA_PROBE_READ_LDS: {
            const size_t lds = (size_t)L * (threads / kWave) * kWave * sizeof(float4);
            if (lds > 64 * 1024) return IQA_ERR_CONFIG;
            return status(launch(&probe_read_lds<L>, blocks, threads, lds, s, src, n4, per,
                                 (int32_t)threads, out));
        }
        default: return IQA_ERR_CONFIG;
    }
}

}  // namespace iqa_probe

using namespace iqa_probe;

extern "C" {

iqa_status iqa_probe_empty(int64_t blocks, int32_t threads, void *stream) {
    if (blocks < 1 || blocks > INT32_MAX || threads < 1 || threads > 1024) return IQA_ERR_SHAPE;
    return status(launch(&probe_empty, (unsigned)blocks, (unsigned)threads, 0,
                         static_cast<hipStream_t>(stream)));
}

iqa_status iqa_probe_read(const float *buf, int64_t n, float *out, int64_t blocks,
                          int32_t threads, int32_t loads, int32_t mode, void *stream) {
    if (!buf || !out) return IQA_ERR_NULL;
    if (n <= 0 || n % 4 != 0 || blocks < 1 || blocks > INT32_MAX) return IQA_ERR_SHAPE;
    if (threads < kWave || threads > 1024 || threads % kWave != 0) return IQA_ERR_CONFIG;
    if (reinterpret_cast<uintptr_t>(buf) % 16 != 0 || reinterpret_cast<uintptr_t>(out) % 4 != 0)
        return IQA_ERR_ALIGN;
    const int64_t n4 = n / 4;
    const int64_t per = (n4 + blocks - 1) / blocks;
    const float4 *src = reinterpret_cast<const float4 *>(buf);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const unsigned b = (unsigned)blocks, t = (unsigned)threads;
    switch (loads) {
        case 4: return read_with<4>(mode, src, n4, per, out, b, t, s);
        case 8: return read_with<8>(mode, src, n4, per, out, b, t, s);
        case 16: return read_with<16>(mode, src, n4, per, out, b, t, s);
        case 32: return read_with<32>(mode, src, n4, per, out, b, t, s);
        default: return IQA_ERR_CONFIG;
    }
}

iqa_status iqa_probe_read_timeline(const float *buf, int64_t n, float *out, int64_t blocks,
                                   int32_t threads, int32_t loads, uint64_t *stamps,
                                   int64_t stamp_count, void *stream) {
    if (!buf || !out || !stamps) return IQA_ERR_NULL;
    if (n <= 0 || n % 4 != 0 || blocks < 1 || blocks > INT32_MAX) return IQA_ERR_SHAPE;
    if (threads < kWave || threads > 1024 || threads % kWave != 0) return IQA_ERR_CONFIG;
    if (stamp_count < 8 * blocks) return IQA_ERR_SHAPE;
    if (reinterpret_cast<uintptr_t>(buf) % 16 != 0 || reinterpret_cast<uintptr_t>(out) % 4 != 0 ||
        reinterpret_cast<uintptr_t>(stamps) % 8 != 0)
        return IQA_ERR_ALIGN;
    const int64_t n4 = n / 4;
    const int64_t per = (n4 + blocks - 1) / blocks;
    const float4 *src = reinterpret_cast<const float4 *>(buf);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const unsigned b = (unsigned)blocks, t = (unsigned)threads;
    const int32_t wd = threads;
    switch (loads) {
        case 4: return status(launch(&probe_read_regs_tl<4>, b, t, 0, s, src, n4, per, wd, out, stamps));
        case 8: return status(launch(&probe_read_regs_tl<8>, b, t, 0, s, src, n4, per, wd, out, stamps));
        case 16: return status(launch(&probe_read_regs_tl<16>, b, t, 0, s, src, n4, per, wd, out, stamps));
        case 32: return status(launch(&probe_read_regs_tl<32>, b, t, 0, s, src, n4, per, wd, out, stamps));
        default: return IQA_ERR_CONFIG;
    }
}

int iqa_probe_last_hip_error(void) { return g_last_error; }

int64_t iqa_wall_clock_khz(void) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return -1;
    return khz;
}

}  // extern "C"
