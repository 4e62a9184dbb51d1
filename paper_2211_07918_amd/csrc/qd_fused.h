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
  int32_t first_gate;              // first member (in circuit order)
  int32_t ngates;                  // number of members
  std::vector<int32_t> members;    // gate indices, ascending
};

// Kernel arguments of the matrix-core block application (by value).
struct FusedArgs {
  float2* psi;
  const float* a32;                 // Kp x Kp real embedding, FP32
  const __bf16* ahi;                // BF16 split
  const __bf16* alo;
  int32_t Kp;                       // leading dimension of the A arrays (64, 128, 192 or 256)
  int32_t twoB;                     // 2B real rows in use
  uint32_t BL, dH, E, NT;           // run length, runs, amplitudes and columns per tile
  uint32_t high_window;             // 1 if no window qudit lies inside a run (column = run offset)
  Magic32 blm;                      // division by BL
  SliceMap tiles;                   // tile index -> global offset of its first run
  const int64_t* hoff;              // dH run offsets from the tile origin
  const int32_t* yh;                // window-local index contributed by each run
  const uint32_t* lmap;             // BL entries: (column << 16) | window-local index part
  const int32_t* rowpos;            // KPAD / 2 entries: tile position of window index y (column 0);
                                    // fill 1: two tables, for a tile origin of even and of odd index
  const int32_t* colpos;            // 16 NTILES entries: tile position of column n (window index 0),
                                    // also its offset in HBM from the start of the run
  const uint32_t* wrow;             // KPAD / 2 entries: HBM offset of amplitude (y, column 0) from
                                    // the tile origin, so (y, n) sits at origin + wrow[y] + colpos[n]
  // How the rows kernel moves a tile between HBM and LDS:
  //   fill 0: even run length, 16-byte units of two amplitudes (every run starts at an even index);
  //   fill 1: odd run length, each run read as (BL + 1) / 2 aligned 16-byte units from the even
  //           index at or below its start, so one spare amplitude per run is read (and never
  //           written back): LDS keeps BL + 1 slots per run, the run at slot offset start & 1;
  //   fill 2: odd run length where a spare read could leave the state's buffer: 4-byte units.
  uint32_t fill;
  uint32_t upr;                     // 16-byte units per run (fill 0, 1)
  Magic32 upm;                      // division by upr
  uint32_t ES;                      // LDS amplitude slots per tile: dH (BL + 1) with fill 1, else E
};

struct FusedBlockDev {
  FusedBlockInfo info{};
  int Kp = 0;                       // padded real dimension (2B rounded up to 32)
  int variant = 0;                  // kernel shape: rows of A per wave and columns per tile
  bool geom_ok = false;
  FusedArgs args{};
  int64_t* tab_hoff = nullptr;
  int32_t* tab_yh = nullptr;
  uint32_t* tab_lmap = nullptr;
  int32_t* tab_rowpos = nullptr;
  int32_t* tab_rowpos_odd = nullptr;   // fill 1 (odd run length): tables for even and odd tile origins
  int32_t* tab_colpos = nullptr;
  uint32_t* tab_wrow = nullptr;
  double* u64 = nullptr;            // B x B complex FP64, row-major interleaved
  float* a32 = nullptr;             // Kp x Kp real embedding, FP32
  __hip_bfloat16* ahi = nullptr;    // BF16 split of a32: hi
  __hip_bfloat16* alo = nullptr;    //                    lo
  std::vector<double> host64;       // host copy of u64
};

int plan_fusion(const Register& r, const qd_gate* gates, int32_t g, int32_t max_block,
                std::vector<int32_t>* block_of, std::vector<FusedBlockInfo>* blocks);
int launch_fused_block(qd_state* s, const struct ::qd_fused* f, int b, int mode);
int fused_geometry(const Register& r, FusedBlockDev* d);
int fused_kpad(int B);            // leading dimension of the real embedding for block dimension B

}  // namespace qd

struct qd_fused {
  qd::Register reg;
  hipStream_t stream = nullptr;
  std::vector<qd::FusedBlockDev> dev;
};
