// tj_select.h - device sketch of the execution-time path selection
// (kernels in tj_select.hip, host side in tj_select.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace tj {

// HyperLogLog with 2^HLL_P registers.
constexpr int HLL_P = 14;
constexpr uint32_t HLL_M = 1u << HLL_P;
constexpr uint32_t HLL_BINS = 64;              // register values 0 .. 64 - HLL_P + 1 (= 51)
constexpr uint32_t HLL_THREADS = 1024;
constexpr uint32_t HLL_MAX_BLOCKS = 512;       // two 64 KiB-LDS blocks per CU
constexpr uint64_t HLL_MIN_ROWS_PER_BLOCK = 16384;
constexpr uint64_t HLL_ROW_ALIGN = 64;         // rows per block are a multiple of this
constexpr uint32_t HLL_GROUPS = 16;            // slab groups of the first merge step
// Blocks (slabs of HLL_M bytes) one column of n rows uses; 0 for n = 0.
uint32_t hll_blocks(uint64_t n);
uint64_t hll_rows_per_block(uint64_t n);
// slab[b][j] = max rank of register j over block b's rows of keys[n].
hipError_t launch_hll_block(int key_bytes, const void* keys, uint64_t n, uint8_t* slab, hipStream_t st);
// regs[3][HLL_M] = R, S and union registers; hist[3][HLL_BINS] = their value
// counts; scratch: part, 2 * HLL_GROUPS * HLL_M bytes, and whist,
// HLL_WHIST_WORDS words.
constexpr uint64_t HLL_WHIST_WORDS = (HLL_M / 64) * 3 * HLL_BINS;
hipError_t launch_hll_finish(const uint8_t* slab_r, uint32_t nb_r, const uint8_t* slab_s, uint32_t nb_s,
                             uint8_t* part, uint8_t* regs, uint32_t* whist, uint32_t* hist, hipStream_t st);

}  // namespace tj
