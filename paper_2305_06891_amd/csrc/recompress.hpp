// Truncated-SVD recompression of ACA factors (see recompress.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace hm {

// Largest rank recompressed (blocks of higher ACA rank keep their factors).
constexpr int RC_KMAX = 256;
constexpr double RC_EARLY = 0.1;

struct RcDev {
  int64_t u_off, v_off;  // FP64 ACA factors in the scratch: U m x k (ld m), V n x k (ld n)
  int64_t w_off;         // workspace offset (doubles), set by recompress_blocks
  int64_t du, dv;        // element offsets of U' (m x r) and V' (n x r) in the stage buffer
  int32_t m, n, k, out;  // out: index of the block's new rank in newrank
  double tol;            // relative truncation tolerance
  // 1: the pivoted Cholesky steps pick the column of largest weighted
  // residual and stop once the discarded columns' weighted residual norms
  // add up to at most RC_EARLY tol |U V^T|_F on each side (a rank-revealing
  // preselection; the block's error stays within (1 + 2 RC_EARLY) tol);
  // 0: every numerically independent column is kept (the exact rule)
  int32_t early = 0, pad = 0;
};

int64_t recompress_work_doubles(int k);

// Recompresses every listed block (2 <= k <= RC_KMAX) and writes its new
// factors to `stage` (FP64 when stage_f64, FP32 otherwise) and its rank r to
// d_newrank[out] (0 for a block whose factors are all zero).  Runs on s and
// synchronises it.
void recompress_blocks(std::vector<RcDev>& blocks, const double* scratch, void* stage, bool stage_f64,
                       int* d_newrank, hipStream_t s);

}  // namespace hm
