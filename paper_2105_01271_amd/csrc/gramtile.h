// Lower 16 x 16 tiles of a Gram X^T X (X up to 128 columns) on the FP64 matrix
// cores, for 256-thread workgroups.  Tile (I, J), I >= J, has the number
// I (I + 1) / 2 + J, so the tiles of an nb-block matrix are 0 .. nb (nb + 1) / 2 - 1
// for every nb; wave w owns tiles w, w + 4, w + 8, ...
//
// MFMA operands for rows r of a block held in LDS (FP64, row stride ld):
// A(i, k) = X(r_k, 16 I + i) in lane i + 16 k, B(k, j) = X(r_k, 16 J + j) in
// lane j + 16 k; the tile entry (i, j) ends in lane j + 16 (i mod 4), register i / 4.
#pragma once

#include "wavechol.h"

namespace gt {

using wc::d4;

constexpr int MAXT = 9;   // tiles per wave: 36 tiles of an 8 x 8 tiling over 4 waves

struct Tiles {
  int ti[MAXT], tj[MAXT];
  int n;
};

__device__ __forceinline__ Tiles tiles_of(int wave, int nb) {
  Tiles s;
  const int ntile = nb * (nb + 1) / 2;
  s.n = 0;
#pragma unroll
  for (int u = 0; u < MAXT; ++u) {
    const int id = wave + 4 * u;
    int I = 0, J = 0;
    if (id < ntile) {
      while ((I + 1) * (I + 2) / 2 <= id) ++I;
      J = id - I * (I + 1) / 2;
      ++s.n;
    }
    s.ti[u] = I;
    s.tj[u] = J;
  }
  return s;
}

__device__ __forceinline__ void zero(d4 (&acc)[MAXT]) {
#pragma unroll
  for (int u = 0; u < MAXT; ++u) acc[u] = d4{0.0, 0.0, 0.0, 0.0};
}

// acc[u] += tile u of rows[0 .. 4 K4) of the LDS block (row stride ld).
template <int K4>
__device__ __forceinline__ void accum(const double *rows, int ld, const Tiles &s, d4 (&acc)[MAXT]) {
  const int lane = threadIdx.x & 63, col = lane & 15, kk = lane >> 4;
#pragma unroll
  for (int k4 = 0; k4 < K4; ++k4) {
    const double *row = rows + (4 * k4 + kk) * ld;
#pragma unroll
    for (int u = 0; u < MAXT; ++u)
      if (u < s.n) acc[u] = wc::mfma(row[16 * s.ti[u] + col], row[16 * s.tj[u] + col], acc[u]);
  }
}

// Tile-major store of this wave's tiles: entry (i, j) of tile id at dst[256 id + 16 i + j].
__device__ __forceinline__ void store_tiles(const d4 (&acc)[MAXT], const Tiles &s, int wave, double *dst) {
  const int lane = threadIdx.x & 63, col = lane & 15, kk = lane >> 4;
#pragma unroll
  for (int u = 0; u < MAXT; ++u) {
    if (u >= s.n) continue;
    const int id = wave + 4 * u;
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[256 * id + (4 * v + kk) * 16 + col] = acc[u][v];
  }
}

}  // namespace gt
