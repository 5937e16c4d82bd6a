// Limits and LDS layout of the symmetric zero-block-omitted SpMV tile:
// shared by the plan builder (which rejects matrices that do not fit and
// marks the entries the kernel must add one lane at a time) and the kernel
// (which sizes its LDS from the plan).
#pragma once
#include <cstddef>

namespace xab {
namespace sym {
constexpr int kRowCap = 2048;          // rows per tile (LDS accumulator of the tile's own rows)
constexpr int kExtCap = 6144;          // LDS slots for column blocks below the tile
constexpr int kLutMax = 2048;          // span of block ids one tile may touch
constexpr int kLutWords = kLutMax / 32;
constexpr int kLdsCap = 65536;         // LDS bytes one symmetric tile may use
constexpr int kLanes = 64;             // one wave per tile
constexpr int kChunkJ = 8;             // entries per lane per chunk
constexpr int kChunk = kLanes * kChunkJ;  // entries per chunk (chunks start at multiples of it)
// bits of the plan's column copy: 31 = first entry of a non-empty row,
// 30 = add this entry's transposed product after the chunk's slots (a
// lower lane of the same slot adds to the same row); columns below 2^30 - 1
constexpr unsigned kHeadBit = 0x80000000u;
constexpr unsigned kDeferBit = 0x40000000u;
constexpr unsigned kColMask = 0x3fffffffu;
constexpr int kMaxCols = (1 << 30) - 1;
// LDS of one tile: accumulators of the own rows and of the touched blocks,
// x of the own rows (accumulation type), the head marks of one chunk and
// the block lookup table
inline constexpr size_t lds_bytes(int own_cap, int ext_cap, int lut_cap, int at_bytes) {
    return (size_t)at_bytes * (2 * (size_t)own_cap + (size_t)ext_cap) + 4 * (size_t)kChunk + 2 * (size_t)lut_cap;
}
// LDS of one tile of the sliced walk: the accumulators, one spare slot per
// lane (the target of the adds that add nothing) and the lookup table
inline constexpr size_t lds_sliced(int own_cap, int ext_cap, int lut_cap, int at_bytes) {
    return (size_t)at_bytes * ((size_t)own_cap + (size_t)ext_cap + kLanes) + 2 * (size_t)lut_cap;
}
// the sliced walk applies when its padding stays within a quarter of the
// entries and no row is longer than 4096 entries (one lane sums a row
// serially: the FP64 product gate of 1e-12 per row holds for far longer)
inline constexpr bool sliced(long long nnz, long long padded, long long widest) {
    return padded <= nnz + nnz / 4 && widest <= 4096;
}
}  // namespace sym
}  // namespace xab
