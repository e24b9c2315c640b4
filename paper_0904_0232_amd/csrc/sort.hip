// Stable tile-major cell sort of the particle slots and compaction of the
// removed ones.  Key = ((tz nTy + ty) nTx + tx) T^3 + (lz T + ly) T + lx with
// (i,j,k) = floor(x); removed particles take the all-ones key of key_bits bits
// and so sort to the end.  The ordering primitive is rocPRIM's stable LSD
// radix sort (through hipCUB) on key_bits bits only; keys, the gather of the
// SoA state and the live count are computed here.
#include <hipcub/hipcub.hpp>

#include "grpic_dev.h"
#include "grpic_impl.h"

namespace grpic {

__global__ void k_sort_keys(Grid G, int T, int nTx, int nTy, uint32_t sentinel, ParticlePtrs in, int64_t n,
                            uint32_t *__restrict__ keys, uint32_t *__restrict__ idx) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    idx[id] = (uint32_t)id;
    if (in.sp[id] == kDead) {
        keys[id] = sentinel;
        return;
    }
    int c[3];
    for (int ax = 0; ax < 3; ax++) {
        int ci = (int)floor(in.x[ax][id]);
        int nn = G.dim(ax);
        c[ax] = ci < 0 ? 0 : (ci > nn - 1 ? nn - 1 : ci);
    }
    uint32_t tx = c[0] / T, ty = c[1] / T, tz = c[2] / T;
    uint32_t lx = c[0] % T, ly = c[1] % T, lz = c[2] % T;
    keys[id] = ((tz * nTy + ty) * nTx + tx) * (uint32_t)(T * T * T) + (lz * T + ly) * T + lx;
}

__global__ void k_sort_gather(ParticlePtrs in, ParticlePtrs out, const uint32_t *__restrict__ idx, int64_t n) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    uint32_t s = idx[id];
    for (int q = 0; q < 3; q++) out.x[q][id] = in.x[q][s];
    for (int q = 0; q < 4; q++) out.u[q][id] = in.u[q][s];
    out.sp[id] = in.sp[s];
}

// live count = position of the first sentinel key
__global__ void k_sort_count(const uint32_t *__restrict__ keys, int64_t n, uint32_t sentinel,
                             unsigned long long *counters) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    bool here = keys[id] == sentinel;
    bool prev = id == 0 ? false : keys[id - 1] == sentinel;
    if (here && !prev) counters[C_NALIVE] = (unsigned long long)id;
    if (id == n - 1 && !here) counters[C_NALIVE] = (unsigned long long)n;
}

size_t sort_temp_bytes(int64_t capacity) {
    size_t bytes = 0;
    hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                       (const uint32_t *)nullptr, (uint32_t *)nullptr, (int)capacity, 0, 32);
    return bytes;
}

void launch_sort(const Grid &G, int tile, int64_t n, ParticlePtrs in, ParticlePtrs out, uint32_t *keys,
                 uint32_t *keys_alt, uint32_t *idx, uint32_t *idx_alt, void *temp, size_t temp_bytes,
                 int key_bits, unsigned long long *counters, hipStream_t s) {
    if (n <= 0) return;
    int nTx = (G.nx + tile - 1) / tile, nTy = (G.ny + tile - 1) / tile;
    uint32_t sentinel = key_bits >= 32 ? 0xFFFFFFFFu : ((1u << key_bits) - 1u);
    unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_sort_keys, dim3(nb), dim3(256), 0, s, G, tile, nTx, nTy, sentinel, in, n, keys, idx);
    size_t tb = temp_bytes;
    hipcub::DeviceRadixSort::SortPairs(temp, tb, keys, keys_alt, idx, idx_alt, (int)n, 0, key_bits, s);
    hipLaunchKernelGGL(k_sort_gather, dim3(nb), dim3(256), 0, s, in, out, idx_alt, n);
    hipLaunchKernelGGL(k_sort_count, dim3(nb), dim3(256), 0, s, keys_alt, n, sentinel, counters);
}

// FP32-mixed: keys from the packed cell.
__global__ void k_sort_keys32(Grid G, int T, int nTx, int nTy, uint32_t sentinel, ParticlePtrs32 in, int64_t n,
                              uint32_t *__restrict__ keys, uint32_t *__restrict__ idx) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    idx[id] = (uint32_t)id;
    if (in.sp[id] == kDead) {
        keys[id] = sentinel;
        return;
    }
    int c[3];
    unpack_cell(in.cell[id], c[0], c[1], c[2]);
    for (int ax = 0; ax < 3; ax++) {
        int nn = G.dim(ax);
        c[ax] = c[ax] < 0 ? 0 : (c[ax] > nn - 1 ? nn - 1 : c[ax]);
    }
    uint32_t tx = c[0] / T, ty = c[1] / T, tz = c[2] / T;
    uint32_t lx = c[0] % T, ly = c[1] % T, lz = c[2] % T;
    keys[id] = ((tz * nTy + ty) * nTx + tx) * (uint32_t)(T * T * T) + (lz * T + ly) * T + lx;
}

__global__ void k_sort_gather32(ParticlePtrs32 in, ParticlePtrs32 out, const uint32_t *__restrict__ idx, int64_t n) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    uint32_t s = idx[id];
    out.cell[id] = in.cell[s];
    for (int q = 0; q < 3; q++) out.off[q][id] = in.off[q][s];
    for (int q = 0; q < 4; q++) out.u[q][id] = in.u[q][s];
    out.sp[id] = in.sp[s];
}

void launch_sort32(const Grid &G, int tile, int64_t n, ParticlePtrs32 in, ParticlePtrs32 out, uint32_t *keys,
                   uint32_t *keys_alt, uint32_t *idx, uint32_t *idx_alt, void *temp, size_t temp_bytes,
                   int key_bits, unsigned long long *counters, hipStream_t s) {
    if (n <= 0) return;
    int nTx = (G.nx + tile - 1) / tile, nTy = (G.ny + tile - 1) / tile;
    uint32_t sentinel = key_bits >= 32 ? 0xFFFFFFFFu : ((1u << key_bits) - 1u);
    unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_sort_keys32, dim3(nb), dim3(256), 0, s, G, tile, nTx, nTy, sentinel, in, n, keys, idx);
    size_t tb = temp_bytes;
    hipcub::DeviceRadixSort::SortPairs(temp, tb, keys, keys_alt, idx, idx_alt, (int)n, 0, key_bits, s);
    hipLaunchKernelGGL(k_sort_gather32, dim3(nb), dim3(256), 0, s, in, out, idx_alt, n);
    hipLaunchKernelGGL(k_sort_count, dim3(nb), dim3(256), 0, s, keys_alt, n, sentinel, counters);
}

}  // namespace grpic
