// Compile-time limits shared by the kernels and the host planning code
// (plain C++: the host planning code also builds without the HIP compiler).
#pragma once

namespace tk {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxBlocks = 4;      // columns per lane: n <= kWave * kMaxBlocks
constexpr int kMaxOrder = 8;       // largest even tensor order instantiated
constexpr int kMaxPoints = kWave * kMaxBlocks;

// Work plan of the Hessian kernels (tk_hess.hip).
constexpr int kHessJT = 16;                  // tile positions per lane
constexpr int kHessL = kHessJT * kWave;      // upper-triangle entries per row tile (at most)
constexpr int kHessItems = 4096;             // target work items of the tile kernel
constexpr int kHessRWaves = 32768;           // target waves of the unit kernel
constexpr int kHessXWaves = 4096;            // target waves of the cross kernel
constexpr int kTB = kMaxOrder + 1;           // binomial table: C(a, b) for b < kTB

}  // namespace tk
