// Constants and helpers shared by the host code and the device code of
// libcsrspmv. Device-only sources include this header (not internal.h), so
// the kernels also compile at run time (the run-time compiler has no host
// standard library).
#pragma once

#include <cstdint>

#include "csrspmv.h"

namespace csr {

constexpr int kBlock = 256;       // threads per workgroup (4 wave64s)
constexpr int kMergeBlock = 64;   // merge-path tile workgroup: one wave64
constexpr int kNumXcd = 8;        // MI355X: 8 accelerator complex dies

// IDX_W8: window codes of row-aligned merge tiles (8-bit rank of the column
// among the tile's distinct columns; the tile's window dictionary maps it back)
// IDX_R8: the same ranks, with each tile's window given as at most
// kRunsMax runs of consecutive columns in a record of kRunWords int32 words
// ([0] the smallest column, [1] entries | runs << 16, [2 + r] run r's first
// column minus [0] | its length << 16), which the tile reads with scalar
// loads before any vector load, so its x window is loaded together with
// the tile's values instead of after a dictionary load
// IDX_W9: window codes with 9-bit ranks on tiles of 1,024 items (IPT 16):
// windows of up to kWideWindowMax entries; the rank's low byte is the code,
// its ninth bit sits in a per-tile record of kWideWords int32 words ([0] the
// entry count, then one 16-bit mask per lane: bit it * VEC + e for the
// lane's element e of load block it)
enum IdxMode { IDX_I32 = 0, IDX_D16 = 1, IDX_D8 = 2, IDX_W8 = 3, IDX_R8 = 4, IDX_W9 = 5 };
constexpr int kWindowMax = 256;  // window entries per tile (8-bit ranks)
constexpr int kWideWindowMax = 512;
constexpr int kWideWords = 1 + 64 / 2;
// Largest nonzero count: indices are int32, and a lane's loop index may step
// up to one workgroup (256) past the last nonzero before it stops, so the
// count keeps that much (and more) below 2^31.
constexpr int64_t kMaxNnz = (int64_t)INT32_MAX - 4095;
constexpr int kRunWords = 16;
constexpr int kRunsMax = kRunWords - 2;

// Logical block of this workgroup in a launch of 8 * per_xcd workgroups:
// workgroups are dispatched to the XCDs round-robin, so logical block
// l = (b % 8) * per_xcd + b / 8 gives every XCD one contiguous range.
__device__ __forceinline__ int64_t xcd_logical_block(int64_t per_xcd) {
    int64_t b = blockIdx.x;
    return (b % kNumXcd) * per_xcd + b / kNumXcd;
}

}  // namespace csr
