// Limits of the symmetric zero-block-omitted SpMV tile: shared by the plan
// builder (which rejects matrices that do not fit) and the kernel (which
// sizes its LDS from the plan).
#pragma once

namespace xab {
namespace sym {
constexpr int kRowCap = 2048;          // rows per tile (LDS accumulator of the tile's own rows)
constexpr int kExtCap = 6144;          // LDS slots for column blocks below the tile
constexpr int kLutMax = 2048;          // span of block ids one tile may touch
constexpr int kLutWords = kLutMax / 32;
constexpr int kLdsCap = 65536;         // LDS bytes one symmetric tile may use
constexpr int kChunkJ = 4;             // entries per lane per chunk
// bytes of the fixed part (head flags of a 256 * kChunkJ chunk + wave totals)
constexpr int kFixedBytes = 256 * kChunkJ * 4 + 4 * 24;
}  // namespace sym
}  // namespace xab
