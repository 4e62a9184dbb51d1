// Fused-block data shared by the fusion builder and the matrix-core apply kernels.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <vector>

#include "qd_internal.h"

namespace qd {

struct FusedBlockInfo {
  int32_t k;                        // window size
  int32_t window[QD_MAX_QUDITS];    // window qudits, ascending (first = most significant)
  int32_t B;                        // block dimension = prod of the window's dims
  int32_t first_gate;
  int32_t ngates;
};

struct FusedBlockDev {
  FusedBlockInfo info{};
  int Kp = 0;                       // padded real dimension (2B rounded up to 16)
  double* u64 = nullptr;            // B x B complex FP64, row-major interleaved
  float* a32 = nullptr;             // Kp x Kp real embedding, FP32
  __hip_bfloat16* ahi = nullptr;    // BF16 split of a32: hi
  __hip_bfloat16* alo = nullptr;    //                    lo
  std::vector<double> host64;       // host copy of u64
};

int plan_fusion(const Register& r, const qd_gate* gates, int32_t g, int32_t max_block,
                std::vector<int32_t>* block_of, std::vector<FusedBlockInfo>* blocks);
int launch_fused_block(qd_state* s, const struct ::qd_fused* f, int b, int mode);

}  // namespace qd

struct qd_fused {
  qd::Register reg;
  hipStream_t stream = nullptr;
  std::vector<qd::FusedBlockDev> dev;
};
