// Per-workgroup LDS copies of the most observed cameras' records.
//
// In point-major order each lane of a wavefront reads the record of its own
// camera, so a 16-byte load of camera words touches up to 64 cache lines and
// costs the L1 one line lookup each; at about one lookup per CU per cycle
// this, not HBM, bounds the kernels that read camera words per observation.
// Cameras are numbered most observed first, so an LDS copy of the records of
// cameras [0, Kc) serves most observations (85% of those of the 29M-
// observation workload with its 900 most observed cameras) without L1
// lookups.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ba {

template <typename T>
using Vec16 = T __attribute__((ext_vector_type(16 / sizeof(T))));

// N words from a 16-byte aligned address: 16 bytes per load, then the
// remainder one word at a time (a load never writes registers it does not
// fill, which would make it wait for older loads into them).
template <typename T, int N>
__device__ __forceinline__ void load_words16(const T* __restrict__ src, T* dst)
{
    constexpr int P = 16 / sizeof(T);
    const Vec16<T>* s = reinterpret_cast<const Vec16<T>*>(src);
#pragma unroll
    for (int c = 0; c < N / P; ++c) {
        const Vec16<T> v = s[c];
#pragma unroll
        for (int e = 0; e < P; ++e) dst[c * P + e] = v[e];
    }
#pragma unroll
    for (int e = N / P * P; e < N; ++e) dst[e] = src[e];
}

// Copies words [0, W) of each of the records [0, Kc) (record stride S words
// in memory) into LDS at stride W, 16 bytes per thread and step; W and S are
// multiples of 16 bytes.  The caller synchronises the workgroup afterwards.
template <typename T, int W, int S, int NT>
__device__ __forceinline__ void fill_camera_cache(const T* __restrict__ src, int32_t Kc, T* cache)
{
    constexpr int RC = W * (int)sizeof(T) / 16, SC = S * (int)sizeof(T) / 16;
    const uint4* s = reinterpret_cast<const uint4*>(src);
    uint4* d = reinterpret_cast<uint4*>(cache);
    for (int q = threadIdx.x; q < Kc * RC; q += NT) {
        const int32_t j = q / RC, c = q - j * RC;
        d[q] = s[(int64_t)j * SC + c];
    }
}

// Words [0, N) of camera j's record: from the LDS copy (stride W) when
// j < Kc, else from memory (stride S).  The LDS reads are issued first: both
// branches fill the same registers, so the memory loads of the other lanes
// wait only for those short reads, never the reverse.
template <typename T, int N, int W, int S>
__device__ __forceinline__ void camera_words(int32_t j, int32_t Kc, const T* cache, const T* __restrict__ src, T* out)
{
    if (j < Kc) load_words16<T, N>(cache + W * j, out);
    __builtin_amdgcn_sched_barrier(0);
    if (j >= Kc)
        load_words16<T, N>(reinterpret_cast<const T*>(reinterpret_cast<const char*>(src) +
                                                      (uint32_t)j * (uint32_t)(S * sizeof(T))),
                           out);
}

}  // namespace ba
