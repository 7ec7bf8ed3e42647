// Home workgroups of a transport round (host side, no HIP types): the round's
// cases hold consecutive chunk ranges [chunk_begin[i], chunk_begin[i + 1]);
// workgroup g of a grid of `grid` workgroups of `waves` waves starts on the
// case holding chunk g * waves (the grid starts on the first chunks in case
// order and moves on through the cases in order).  Case i's home workgroups
// are [wg_lo[i], wg_lo[i + 1]) (the last ends at grid; a case may have none),
// and their home_waves[i] waves take the case's first chunks by rank.
#pragma once

#include <algorithm>
#include <cstdint>

namespace ctd {

inline void home_workgroups(const uint64_t *chunk_begin, int nrc, int grid, int waves,
                            uint32_t *wg_lo, uint32_t *home_waves) {
  auto first_wg = [&](uint64_t chunk) {  // first g with g * waves >= chunk, at most grid
    const uint64_t g = (chunk + (uint64_t)waves - 1) / (uint64_t)waves;
    return (uint32_t)std::min<uint64_t>(g, (uint64_t)grid);
  };
  for (int i = 0; i < nrc; ++i) wg_lo[i] = first_wg(chunk_begin[i]);
  for (int i = 0; i < nrc; ++i) {
    const uint32_t hi = i + 1 < nrc ? wg_lo[i + 1] : (uint32_t)grid;
    home_waves[i] = (hi - wg_lo[i]) * (uint32_t)waves;
  }
}

}  // namespace ctd
