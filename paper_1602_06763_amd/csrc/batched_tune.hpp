// Per-size-bucket choices of the batched factorizations: the crossover of
// each matrix's recursion (Cholesky: potf2 leaf 32 or 64; LU: panel width 16
// or 32) and the edge of the workgroup's matrix-core product tiles (32 or 64),
// for the buckets n <= 64, <= 128, <= 256 and above. Each matrix's recursion
// itself stays free of tuning (splits at n/2, rounded to 64); only these two
// sizes are chosen per bucket.
//
// Written by paper_1602_06763_amd/autotune.py on AMD Radeon Graphics, 2026-12-03: one batched call
// of 3000 matrices per bucket (sizes uniform over the bucket), median time per
// candidate; the fastest is kept.
//   dpotrf n in [8, 64] leaf 32 tile 32: 0.212 ms
//   dpotrf n in [8, 64] leaf 32 tile 64: 0.221 ms
//   dpotrf n in [8, 64] leaf 64 tile 32: 0.164 ms
//   dpotrf n in [8, 64] leaf 64 tile 64: 0.161 ms
//   dpotrf n in [65, 128] leaf 32 tile 32: 0.691 ms
//   dpotrf n in [65, 128] leaf 32 tile 64: 0.687 ms
//   dpotrf n in [65, 128] leaf 64 tile 32: 0.518 ms
//   dpotrf n in [65, 128] leaf 64 tile 64: 0.490 ms
//   dpotrf n in [129, 256] leaf 32 tile 32: 2.088 ms
//   dpotrf n in [129, 256] leaf 32 tile 64: 1.992 ms
//   dpotrf n in [129, 256] leaf 64 tile 32: 1.777 ms
//   dpotrf n in [129, 256] leaf 64 tile 64: 1.617 ms
//   dpotrf n in [257, 512] leaf 32 tile 32: 9.810 ms
//   dpotrf n in [257, 512] leaf 32 tile 64: 7.911 ms
//   dpotrf n in [257, 512] leaf 64 tile 32: 9.216 ms
//   dpotrf n in [257, 512] leaf 64 tile 64: 7.165 ms
//   spotrf n in [8, 64] leaf 32 tile 32: 0.177 ms
//   spotrf n in [8, 64] leaf 32 tile 64: 0.179 ms
//   spotrf n in [8, 64] leaf 64 tile 32: 0.142 ms
//   spotrf n in [8, 64] leaf 64 tile 64: 0.140 ms
//   spotrf n in [65, 128] leaf 32 tile 32: 0.532 ms
//   spotrf n in [65, 128] leaf 32 tile 64: 0.516 ms
//   spotrf n in [65, 128] leaf 64 tile 32: 0.390 ms
//   spotrf n in [65, 128] leaf 64 tile 64: 0.356 ms
//   spotrf n in [129, 256] leaf 32 tile 32: 1.609 ms
//   spotrf n in [129, 256] leaf 32 tile 64: 1.458 ms
//   spotrf n in [129, 256] leaf 64 tile 32: 1.365 ms
//   spotrf n in [129, 256] leaf 64 tile 64: 1.175 ms
//   spotrf n in [257, 512] leaf 32 tile 32: 7.646 ms
//   spotrf n in [257, 512] leaf 32 tile 64: 5.583 ms
//   spotrf n in [257, 512] leaf 64 tile 32: 7.211 ms
//   spotrf n in [257, 512] leaf 64 tile 64: 5.087 ms
//   dgetrf n in [8, 64] leaf 16 tile 32: 0.677 ms
//   dgetrf n in [8, 64] leaf 16 tile 64: 0.686 ms
//   dgetrf n in [8, 64] leaf 32 tile 32: 0.558 ms
//   dgetrf n in [8, 64] leaf 32 tile 64: 0.569 ms
//   dgetrf n in [65, 128] leaf 16 tile 32: 2.229 ms
//   dgetrf n in [65, 128] leaf 16 tile 64: 2.212 ms
//   dgetrf n in [65, 128] leaf 32 tile 32: 1.774 ms
//   dgetrf n in [65, 128] leaf 32 tile 64: 1.757 ms
//   dgetrf n in [129, 256] leaf 16 tile 32: 6.544 ms
//   dgetrf n in [129, 256] leaf 16 tile 64: 6.170 ms
//   dgetrf n in [129, 256] leaf 32 tile 32: 5.170 ms
//   dgetrf n in [129, 256] leaf 32 tile 64: 4.772 ms
//   sgetrf n in [8, 64] leaf 16 tile 32: 0.494 ms
//   sgetrf n in [8, 64] leaf 16 tile 64: 0.495 ms
//   sgetrf n in [8, 64] leaf 32 tile 32: 0.400 ms
//   sgetrf n in [8, 64] leaf 32 tile 64: 0.406 ms
//   sgetrf n in [65, 128] leaf 16 tile 32: 1.620 ms
//   sgetrf n in [65, 128] leaf 16 tile 64: 1.557 ms
//   sgetrf n in [65, 128] leaf 32 tile 32: 1.264 ms
//   sgetrf n in [65, 128] leaf 32 tile 64: 1.229 ms
//   sgetrf n in [129, 256] leaf 16 tile 32: 4.762 ms
//   sgetrf n in [129, 256] leaf 16 tile 64: 4.327 ms
//   sgetrf n in [129, 256] leaf 32 tile 32: 3.737 ms
//   sgetrf n in [129, 256] leaf 32 tile 64: 3.353 ms
#pragma once

namespace rl {

constexpr int kBatchBuckets = 4;
__host__ __device__ constexpr int batch_bucket(int n) { return n <= 64 ? 0 : n <= 128 ? 1 : n <= 256 ? 2 : 3; }

struct BatchTune {
    unsigned char leaf[kBatchBuckets];
    unsigned char tile[kBatchBuckets];
};

// routines: dpotrf, spotrf, dgetrf, sgetrf
constexpr BatchTune kTuneDefault[4] = {
    {{64, 64, 64, 64}, {64, 64, 64, 64}},   // dpotrf
    {{64, 64, 64, 64}, {64, 64, 64, 64}},   // spotrf
    {{32, 32, 32, 32}, {32, 64, 64, 64}},   // dgetrf
    {{32, 32, 32, 32}, {32, 64, 64, 64}},   // sgetrf
};

}  // namespace rl
