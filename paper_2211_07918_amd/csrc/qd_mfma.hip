// Application of fused B x B blocks to a complex64 state on the gfx950 matrix cores.
//
// Every slice of the state over a block's window (the B amplitudes that share all other digits)
// is one column of X; the block acts as Y = U X. The complex product runs as a real one:
// with interleaved rows (2y + c, c = re/im) U becomes the real matrix A of 2x2 blocks
// [[Re u, -Im u], [Im u, Re u]] and X the real (2B) x N matrix of the slices' (re, im) parts.
//
// A workgroup (4 waves) owns tiles of the state: dH runs of BL contiguous amplitudes, the low
// suffix of the register (BL) times the window qudits above it (dH), i.e. NT = BL dH / B whole
// columns. Per tile: coalesced loads of the runs scattered into LDS as X[n][k] (k = 2y + c),
// MFMA accumulation with each wave holding its rows of A in registers for the whole launch,
// results written back to LDS and stored with the same coalesced runs.
//   FP32 mode:  v_mfma_f32_16x16x4_f32, FP32 accumulation.
//   BF16x3 mode: a = a_hi + a_lo, x = x_hi + x_lo in BF16; a_hi x_hi + a_hi x_lo + a_lo x_hi with
//               v_mfma_f32_16x16x32_bf16 and FP32 accumulation (the a_lo x_lo term is dropped).
// Operand layouts (lane l of 64): 16x16x4 f32: A[l%16][l/16], B[l/16][l%16];
// 16x16x32 bf16: A[l%16][8(l/16)+j], B[8(l/16)+j][l%16]; result D[4(l/16)+i][l%16].
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>

#include "qd_fused.h"
#include "qd_stream.h"

namespace qd {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ int64_t fm_offset(const SliceMap& sm, uint32_t idx) {
  int64_t off = sm.base;
  uint32_t rem = idx;
#pragma unroll
  for (int g = 0; g < kMaxGroups; ++g) {
    if (g < int(sm.ng)) {
      const uint32_t q = (g + 1 < int(sm.ng)) ? magic_div(rem, sm.gmag[g]) : 0u;
      const uint32_t r = rem - q * sm.gdim[g];
      off += int64_t(r) * sm.gstride[g];
      rem = q;
    }
  }
  return off;
}

// Column and window-local row of tile amplitude e (run h = e / BL, offset lo inside the run).
__device__ __forceinline__ void tile_coords(const FusedArgs& a, const int32_t* s_yh, uint32_t e, uint32_t* h,
                                            uint32_t* lo, uint32_t* n, uint32_t* y) {
  *h = magic_div(e, a.blm);
  *lo = e - *h * a.BL;
  if (a.high_window) {  // no window qudit inside the run: the run offset is the column
    *n = *lo;
    *y = uint32_t(s_yh[*h]);
  } else {
    const uint32_t lm = a.lmap[*lo];
    *n = lm >> 16;
    *y = uint32_t(s_yh[*h]) + (lm & 0xFFFFu);
  }
}

// Moves the E amplitudes of a tile between HBM and the LDS column layout X[n][2y + c]
// (TO_LDS: HBM -> LDS). A thread holds 2 CH amplitudes in flight: every HBM access of a pass is
// issued before the first LDS access that depends on it. With an even run length a unit is two
// adjacent amplitudes (one 16-byte access), else one amplitude (8 bytes).
template <bool TO_LDS, int CH>
__device__ __forceinline__ void tile_move(const FusedArgs& a, float2* __restrict__ psi, float* xs, uint32_t P,
                                          const int64_t* s_hoff, const int32_t* s_yh, int64_t g0) {
  constexpr int S = 2 * CH;
  const uint32_t tid = threadIdx.x;
  float sr[S], si[S];
  if ((a.BL & 1u) == 0) {
    const uint32_t units = a.E >> 1;
    for (uint32_t base = 0; base < units; base += 256 * CH) {
      if (!TO_LDS) {
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          const uint32_t u = base + tid + 256 * j;
          if (u < units) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              uint32_t h, lo, n, y;
              tile_coords(a, s_yh, 2 * u + q, &h, &lo, &n, &y);
              const float2 t = *reinterpret_cast<const float2*>(xs + n * P + 2 * y);
              sr[2 * j + q] = t.x;
              si[2 * j + q] = t.y;
            }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const uint32_t u = base + tid + 256 * j;
        if (u < units) {
          const uint32_t e = 2 * u;
          const uint32_t h = magic_div(e, a.blm);
          float4* g = reinterpret_cast<float4*>(psi + (g0 + s_hoff[h] + (e - h * a.BL)));
          if (TO_LDS) {
            const float4 t = *g;
            sr[2 * j] = t.x; si[2 * j] = t.y; sr[2 * j + 1] = t.z; si[2 * j + 1] = t.w;
          } else {
            float4 t;
            t.x = sr[2 * j]; t.y = si[2 * j]; t.z = sr[2 * j + 1]; t.w = si[2 * j + 1];
            *g = t;
          }
        }
      }
      if (TO_LDS) {
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          const uint32_t u = base + tid + 256 * j;
          if (u < units) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              uint32_t h, lo, n, y;
              tile_coords(a, s_yh, 2 * u + q, &h, &lo, &n, &y);
              float2 t;
              t.x = sr[2 * j + q];
              t.y = si[2 * j + q];
              *reinterpret_cast<float2*>(xs + n * P + 2 * y) = t;
            }
          }
        }
      }
    }
    return;
  }
  const uint32_t units = a.E;
  for (uint32_t base = 0; base < units; base += 256 * S) {
    if (!TO_LDS) {
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const uint32_t u = base + tid + 256 * k;
        if (u < units) {
          uint32_t h, lo, n, y;
          tile_coords(a, s_yh, u, &h, &lo, &n, &y);
          const float2 t = *reinterpret_cast<const float2*>(xs + n * P + 2 * y);
          sr[k] = t.x;
          si[k] = t.y;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < S; ++k) {
      const uint32_t u = base + tid + 256 * k;
      if (u < units) {
        const uint32_t h = magic_div(u, a.blm);
        float2* g = psi + (g0 + s_hoff[h] + (u - h * a.BL));
        if (TO_LDS) {
          const float2 t = *g;
          sr[k] = t.x;
          si[k] = t.y;
        } else {
          float2 t;
          t.x = sr[k];
          t.y = si[k];
          *g = t;
        }
      }
    }
    if (TO_LDS) {
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const uint32_t u = base + tid + 256 * k;
        if (u < units) {
          uint32_t h, lo, n, y;
          tile_coords(a, s_yh, u, &h, &lo, &n, &y);
          float2 t;
          t.x = sr[k];
          t.y = si[k];
          *reinterpret_cast<float2*>(xs + n * P + 2 * y) = t;
        }
      }
    }
  }
}

// MTW: 16-row tiles of A per wave (4 waves cover KPAD = 64 MTW rows); NTILES: 16-column tiles of
// X per tile of the state; KS: K steps (4 reals each in FP32, 32 in BF16). A is stored KPAD x KPAD
// with zeros beyond 2B, so the hot loop carries no bounds test.
template <int MTW, int NTILES, int KS, bool BF>
__global__ __launch_bounds__(256) void k_fused(FusedArgs a) {
  constexpr int KPAD = 64 * MTW;
  constexpr int P = KPAD + 4;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  float* xs = reinterpret_cast<float*>(lds_raw);
  constexpr uint32_t xs_floats = uint32_t(NTILES) * 16u * P;
  int64_t* s_hoff = reinterpret_cast<int64_t*>(xs + xs_floats);
  int32_t* s_yh = reinterpret_cast<int32_t*>(s_hoff + a.dH);
  float2* __restrict__ psi = a.psi;
  const uint32_t tid = threadIdx.x, w = tid >> 6, l = tid & 63;

  for (uint32_t i = tid; i < xs_floats; i += 256) xs[i] = 0.f;  // padded rows stay zero
  for (uint32_t h = tid; h < a.dH; h += 256) {
    s_hoff[h] = a.hoff[h];
    s_yh[h] = a.yh[h];
  }

  // this wave's rows of A (M-tiles w, w + 4, ...) as MFMA A-operands, for the whole launch
  float af[BF ? 1 : MTW][BF ? 1 : KS];
  v8bf ahi[BF ? MTW : 1][BF ? KS : 1], alo[BF ? MTW : 1][BF ? KS : 1];
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
    const int row = 16 * (int(w) + 4 * i) + int(l & 15);
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      if constexpr (BF) {
        const int k0 = 32 * kk + 8 * int(l >> 4);
        ahi[i][kk] = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(a.ahi + size_t(row) * KPAD + k0));
        alo[i][kk] = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(a.alo + size_t(row) * KPAD + k0));
      } else {
        af[i][kk] = a.a32[size_t(row) * KPAD + 4 * kk + (l >> 4)];
      }
    }
  }
  __syncthreads();

  for (uint32_t tile = blockIdx.x; tile < a.tiles.count; tile += gridDim.x) {
    const int64_t g0 = fm_offset(a.tiles, tile);
    tile_move<true, (512 * NTILES * MTW + 511) / 512>(a, psi, xs, P, s_hoff, s_yh, g0);
    __syncthreads();

    v4f acc[MTW][NTILES];
#pragma unroll
    for (int i = 0; i < MTW; ++i)
#pragma unroll
      for (int nt = 0; nt < NTILES; ++nt) acc[i][nt] = v4f{0.f, 0.f, 0.f, 0.f};

#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
#pragma unroll
      for (int nt = 0; nt < NTILES; ++nt) {
        const float* col = xs + (16 * nt + (l & 15)) * P;
        if constexpr (BF) {
          const float4 x0 = *reinterpret_cast<const float4*>(col + 32 * kk + 8 * (l >> 4));
          const float4 x1 = *reinterpret_cast<const float4*>(col + 32 * kk + 8 * (l >> 4) + 4);
          const float xv[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
          v8bf bh, bl;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const __bf16 hj = (__bf16)xv[j];
            bh[j] = hj;
            bl[j] = (__bf16)(xv[j] - (float)hj);
          }
#pragma unroll
          for (int i = 0; i < MTW; ++i) {
            v4f c = acc[i][nt];
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[i][kk], bh, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[i][kk], bl, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[i][kk], bh, c, 0, 0, 0);
            acc[i][nt] = c;
          }
        } else {
          const float b = col[4 * kk + (l >> 4)];
#pragma unroll
          for (int i = 0; i < MTW; ++i)
            acc[i][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][kk], b, acc[i][nt], 0, 0, 0);
        }
      }
    }
    __syncthreads();  // every wave has read X
#pragma unroll
    for (int i = 0; i < MTW; ++i) {
#pragma unroll
      for (int nt = 0; nt < NTILES; ++nt) {
        float* col = xs + (16 * nt + (l & 15)) * P + 16 * (int(w) + 4 * i) + 4 * (l >> 4);
#pragma unroll
        for (int r = 0; r < 4; ++r) col[r] = acc[i][nt][r];
      }
    }
    __syncthreads();
    tile_move<false, (512 * NTILES * MTW + 511) / 512>(a, psi, xs, P, s_hoff, s_yh, g0);
    __syncthreads();
  }
}

// The tile stays in LDS in its HBM order (run h, offset lo): amplitude (window index y, column n)
// sits at rowpos[y] + colpos[n], because the tile index is linear in the digits (window digits
// give rowpos, the other digits of the run give colpos). The fill is a direct HBM -> LDS copy
// (global_load_lds: no registers, every access of the tile in flight), each lane keeps the column
// offsets of its MFMA operands in registers and reads the row offsets from LDS, and the drain goes
// through registers in batches. Padding rows (y >= B) alias row 0 and padding columns column 0:
// the padded columns of A are zero and a result column depends on its own operand column only.
// NH: passes over K per tile, each over NTILES / NH column tiles (fewer accumulators, so two
// workgroups share a CU and one's copies overlap the other's products). WPE: waves per SIMD the
// register allocation must allow.
constexpr uint32_t kRowsSlack = 256;
constexpr int kNt = 2;   // cache policy of the tile copies: nontemporal (the state streams through)
constexpr size_t kLdsBytes = 160 * 1024;   // floats after a tile: overshoot of the last 64-lane copy

__host__ __device__ inline uint32_t rows_buf_floats(uint32_t E) { return (2u * E + kRowsSlack + 3u) & ~3u; }

// LEFT (FP32): the tile's last column tile holds one column only (81 columns in 6 tiles of 16). Its
// MFMA products are skipped; that column is computed on the vector units from the A rows each lane
// already holds, the four lanes of a row summed by wavefront shuffles.
template <int MTW, int NTILES, int NH, int KS, bool BF, int WPE, int FILL, bool LEFT>
__global__ __launch_bounds__(256, WPE) void k_fused_rows(FusedArgs a) {
  constexpr int KPAD = 64 * MTW;
  constexpr int RY = KPAD / 2;
  constexpr int NTH = NTILES / NH;   // column tiles per pass over K
  static_assert(NTILES % NH == 0, "column tiles split evenly");
  extern __shared__ __align__(16) unsigned char lds_raw[];
  float* xs = reinterpret_cast<float*>(lds_raw);
  int32_t* s_rowpos = reinterpret_cast<int32_t*>(xs + rows_buf_floats(a.ES));
  int64_t* s_hoff = reinterpret_cast<int64_t*>(s_rowpos + 2 * RY);
  uint32_t* xw = reinterpret_cast<uint32_t*>(xs);   // BF16x3: amplitude e holds (hi, lo) at words 2e, 2e + 1
  float2* __restrict__ psi = a.psi;
  const uint32_t tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const uint32_t nrow = FILL == 1 ? 2u * RY : uint32_t(RY);

  for (uint32_t h = tid; h < a.dH; h += 256) s_hoff[h] = a.hoff[h];
  for (uint32_t y = tid; y < nrow; y += 256) s_rowpos[y] = a.rowpos[y];
  // tile-local amplitude index of this lane's column in each column tile
  int32_t cp[NTILES];
#pragma unroll
  for (int nt = 0; nt < NTILES; ++nt) cp[nt] = a.colpos[16 * nt + (l & 15)];

  float af[BF ? 1 : MTW][BF ? 1 : KS];
  v8bf ahi[BF ? MTW : 1][BF ? KS : 1], alo[BF ? MTW : 1][BF ? KS : 1];
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
    const int row = 16 * (int(w) + 4 * i) + int(l & 15);
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      if constexpr (BF) {
        const int k0 = 32 * kk + 8 * int(l >> 4);
        ahi[i][kk] = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(a.ahi + size_t(row) * KPAD + k0));
        alo[i][kk] = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(a.alo + size_t(row) * KPAD + k0));
      } else {
        af[i][kk] = a.a32[size_t(row) * KPAD + 2 * (4 * (kk >> 1) + int(l >> 4)) + (kk & 1)];
      }
    }
  }
  __syncthreads();

  constexpr uint32_t odd = FILL == 1 ? 1u : 0u;
  const uint32_t E = a.E, ES = a.ES;
  // global amplitude index (below 2^32 on this path) of the first amplitude of 16-byte unit u of the
  // tile whose origin is g0 (with fill 1 the unit may start one amplitude before its run, or end
  // one after it); lo0: the offset of that amplitude inside its run
  auto unit_addr = [&](uint32_t g0, uint32_t u, int32_t* lo0) -> uint32_t {
    const uint32_t h = magic_div(u, a.upm), k = u - h * a.upr;
    const uint32_t start = g0 + uint32_t(s_hoff[h]);
    const uint32_t par = start & odd;
    *lo0 = int32_t(2 * k) - int32_t(par);
    return start - par + 2 * k;
  };
  for (uint32_t tile = blockIdx.x; tile < a.tiles.count; tile += gridDim.x) {
    const int64_t g0 = fm_offset(a.tiles, tile);
    const int32_t* rows = FILL == 1 ? s_rowpos + RY * (uint32_t(g0) & 1u) : s_rowpos;
    // ---- fill: LDS float f of the tile <- the amplitude's part in HBM (lane-consecutive LDS).
    // Batches of 8 copies per wave without bounds tests, so their run-offset lookups overlap.
    if constexpr (FILL == 0) {
      const uint32_t units = E >> 1;  // 16 bytes: two adjacent amplitudes of one run
      uint32_t u0 = w * 64;
      for (; u0 + 256 * 7 + 64 <= units; u0 += 256 * 8) {
        int64_t ho[8];
        uint32_t lo[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const uint32_t e = 2 * (u0 + 256 * j + l), h = magic_div(e, a.blm);
          ho[j] = s_hoff[h];
          lo[j] = e - h * a.BL;
        }
        __builtin_amdgcn_sched_barrier(0);   // the 8 lookups are in flight together
#pragma unroll
        for (int j = 0; j < 8; ++j)
          __builtin_amdgcn_global_load_lds(psi + (g0 + ho[j] + lo[j]), xs + 4 * (u0 + 256 * j), 16, 0, kNt);
      }
      for (; u0 < units; u0 += 256) {
        const uint32_t u = u0 + l;
        const float2* src = psi + g0;
        if (u < units) {
          const uint32_t e = 2 * u, h = magic_div(e, a.blm);
          src = psi + (g0 + s_hoff[h] + (e - h * a.BL));
        }
        __builtin_amdgcn_global_load_lds(src, xs + 4 * u0, 16, 0, kNt);
      }
    } else if constexpr (FILL == 1) {
      const uint32_t units = ES >> 1;  // 16 bytes: two adjacent amplitudes, 16-byte aligned
      uint32_t u0 = w * 64;
      for (; u0 + 256 * 7 + 64 <= units; u0 += 256 * 8) {
        uint32_t ga[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          int32_t lo0;
          ga[j] = unit_addr(uint32_t(g0), u0 + 256 * j + l, &lo0);
        }
        __builtin_amdgcn_sched_barrier(0);   // the 8 lookups are in flight together
#pragma unroll
        for (int j = 0; j < 8; ++j) __builtin_amdgcn_global_load_lds(psi + ga[j], xs + 4 * (u0 + 256 * j), 16, 0, kNt);
      }
      for (; u0 < units; u0 += 256) {
        const uint32_t u = u0 + l;
        const float2* src = psi + (uint32_t(g0) - (uint32_t(g0) & odd));
        if (u < units) {
          int32_t lo0;
          src = psi + unit_addr(uint32_t(g0), u, &lo0);
        }
        __builtin_amdgcn_global_load_lds(src, xs + 4 * u0, 16, 0, kNt);
      }
    } else {
      const uint32_t units = E * 2;   // 4 bytes: one part of one amplitude
      const float* pf = reinterpret_cast<const float*>(psi);
      uint32_t u0 = w * 64;
      for (; u0 + 256 * 7 + 64 <= units; u0 += 256 * 8) {
        int64_t ho[8];
        uint32_t lo[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const uint32_t f = u0 + 256 * j + l, e = f >> 1, h = magic_div(e, a.blm);
          ho[j] = s_hoff[h];
          lo[j] = 2 * (e - h * a.BL) + (f & 1u);
        }
        __builtin_amdgcn_sched_barrier(0);   // the 8 lookups are in flight together
#pragma unroll
        for (int j = 0; j < 8; ++j)
          __builtin_amdgcn_global_load_lds(pf + (2 * (g0 + ho[j]) + lo[j]), xs + u0 + 256 * j, 4, 0, kNt);
      }
      for (; u0 < units; u0 += 256) {
        const uint32_t f = u0 + l;
        const float* src = pf + 2 * g0;
        if (f < units) {
          const uint32_t e = f >> 1, h = magic_div(e, a.blm);
          src = pf + 2 * (g0 + s_hoff[h] + (e - h * a.BL)) + (f & 1u);
        }
        __builtin_amdgcn_global_load_lds(src, xs + u0, 4, 0, kNt);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    if constexpr (BF) {
      // split every amplitude once, x = hi + lo in BF16, in place: (re, im) pairs of hi, then of lo
      auto split1 = [&](uint32_t e) {
        const float2 v = *reinterpret_cast<const float2*>(xs + 2 * e);
        const __bf16 hr = (__bf16)v.x, hi = (__bf16)v.y;
        const __bf16 lr = (__bf16)(v.x - (float)hr), li = (__bf16)(v.y - (float)hi);
        uint2 o;
        o.x = uint32_t(__builtin_bit_cast(uint16_t, hr)) | (uint32_t(__builtin_bit_cast(uint16_t, hi)) << 16);
        o.y = uint32_t(__builtin_bit_cast(uint16_t, lr)) | (uint32_t(__builtin_bit_cast(uint16_t, li)) << 16);
        *reinterpret_cast<uint2*>(xw + 2 * e) = o;
      };
      uint32_t base = 0;
      for (; base + 256 * 4 <= ES; base += 256 * 4) {
#pragma unroll
        for (int j = 0; j < 4; ++j) split1(base + tid + 256 * j);
      }
      for (uint32_t e = base + tid; e < ES; e += 256) split1(e);
      __syncthreads();
    }

#pragma unroll
    for (int hf = 0; hf < NH; ++hf) {
      v4f acc[MTW][NTH];
#pragma unroll
      for (int i = 0; i < MTW; ++i)
#pragma unroll
        for (int t = 0; t < NTH; ++t) acc[i][t] = v4f{0.f, 0.f, 0.f, 0.f};

      if constexpr (BF) {
        // lane: column n = 16 nt + (l & 15), rows y = 16 kk + 4 (l >> 4) + q, q = 0..3 (both parts).
        // Operand group g = (kk, t) is loaded one group ahead of its products (scheduling barriers
        // keep that order); the rows of K step kk + 1 are read at the start of K step kk.
        constexpr int G = KS * NTH;
        const int32_t* rpl = rows + 4 * (l >> 4);
        int4 rq[2];
        rq[0] = *reinterpret_cast<const int4*>(rpl);
        uint4 oh[2], ol[2];
        auto load_group = [&](int g) {
          const int kk = g / NTH, nt = hf * NTH + g % NTH;
          const int4 r = rq[kk & 1];
          const int c = cp[nt];
          uint4 h, lo;
          h.x = xw[2 * (r.x + c)]; h.y = xw[2 * (r.y + c)]; h.z = xw[2 * (r.z + c)]; h.w = xw[2 * (r.w + c)];
          lo.x = xw[2 * (r.x + c) + 1]; lo.y = xw[2 * (r.y + c) + 1];
          lo.z = xw[2 * (r.z + c) + 1]; lo.w = xw[2 * (r.w + c) + 1];
          oh[g & 1] = h;
          ol[g & 1] = lo;
        };
        load_group(0);
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int kk = g / NTH, t = g % NTH;
          if (t == 0 && kk + 1 < KS) rq[(kk + 1) & 1] = *reinterpret_cast<const int4*>(rpl + 16 * (kk + 1));
          if (g + 1 < G) load_group(g + 1);
          __builtin_amdgcn_sched_barrier(0);
          const v8bf bh = __builtin_bit_cast(v8bf, oh[g & 1]);
          const v8bf bl = __builtin_bit_cast(v8bf, ol[g & 1]);
          if (!(LEFT && hf == NH - 1 && t == NTH - 1)) {
#pragma unroll
            for (int i = 0; i < MTW; ++i) {
              v4f c = acc[i][t];
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[i][kk], bh, c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[i][kk], bl, c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[i][kk], bh, c, 0, 0, 0);
              acc[i][t] = c;
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      } else {
        // K in pairs of steps: in steps 2 j and 2 j + 1 lane l takes the real and the imaginary
        // part of amplitude (row y = 4 j + (l >> 4), column n = 16 nt + (l & 15)), one 8-byte LDS
        // read for two products. The operands of pair j + 1 are loaded before the products of
        // pair j (scheduling barriers keep that order).
        static_assert(KS % 2 == 0, "K steps in pairs");
        constexpr int KP = KS / 2;
        const float2* x2 = reinterpret_cast<const float2*>(xs);
        const int32_t* rpl = rows + (l >> 4);
        float2 b[2][NTH];
        int32_t rk = rpl[0];
#pragma unroll
        for (int t = 0; t < NTH; ++t) b[0][t] = x2[rk + cp[hf * NTH + t]];
        rk = rpl[4];
#pragma unroll
        for (int j = 0; j < KP; ++j) {
          if (j + 1 < KP) {
#pragma unroll
            for (int t = 0; t < NTH; ++t) b[(j + 1) & 1][t] = x2[rk + cp[hf * NTH + t]];
            if (j + 2 < KP) rk = rpl[4 * (j + 2)];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int t = 0; t < NTH; ++t)
            if (!(LEFT && hf == NH - 1 && t == NTH - 1)) {
#pragma unroll
              for (int i = 0; i < MTW; ++i) {
                acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][2 * j], b[j & 1][t].x, acc[i][t], 0, 0, 0);
                acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][2 * j + 1], b[j & 1][t].y, acc[i][t], 0, 0, 0);
              }
            }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      __syncthreads();  // every wave has read the operands of these columns
      // results of these columns over their own operands (other columns are not touched)
#pragma unroll
      for (int i = 0; i < MTW; ++i) {
        const uint32_t y0 = 8 * (w + 4 * i) + 2 * (l >> 4);   // result rows 2 y0 .. 2 y0 + 3
        const int32_t r0 = 2 * rows[y0], r1 = 2 * rows[y0 + 1];
#pragma unroll
        for (int t = 0; t < NTH; ++t) {
          const int nt = hf * NTH + t;
          const uint32_t n = 16 * nt + (l & 15);
          if (!(LEFT && nt == NTILES - 1) && n < a.NT) {
            float2 v;
            if (y0 < uint32_t(a.twoB / 2)) {
              v.x = acc[i][t][0];
              v.y = acc[i][t][1];
              *reinterpret_cast<float2*>(xs + r0 + 2 * cp[nt]) = v;
            }
            if (y0 + 1 < uint32_t(a.twoB / 2)) {
              v.x = acc[i][t][2];
              v.y = acc[i][t][3];
              *reinterpret_cast<float2*>(xs + r1 + 2 * cp[nt]) = v;
            }
          }
        }
      }
    }
    __syncthreads();
    if constexpr (LEFT) {
      // the single column of the last column tile: lane (row r = 16 (w + 4 i) + (l & 15)) sums
      // A[r][k] x[k] over its own k (those of its A registers), then the four lanes of the row
      const int32_t cl = a.colpos[16 * (NTILES - 1)];
      float part[MTW];
#pragma unroll
      for (int i = 0; i < MTW; ++i) part[i] = 0.f;
      static_assert(!BF, "the single-column path is FP32 only");
      const float2* x2 = reinterpret_cast<const float2*>(xs);
#pragma unroll
      for (int j = 0; j < KS / 2; ++j) {   // complex row 4 j + (l >> 4): real rows 2 (4 j + (l >> 4)) + c
        const float2 x = x2[rows[4 * j + int(l >> 4)] + cl];
#pragma unroll
        for (int i = 0; i < MTW; ++i) part[i] = fmaf(af[i][2 * j + 1], x.y, fmaf(af[i][2 * j], x.x, part[i]));
      }
#pragma unroll
      for (int i = 0; i < MTW; ++i) {
        part[i] += __shfl_xor(part[i], 16);
        part[i] += __shfl_xor(part[i], 32);
      }
      __syncthreads();   // every wave has read the column
      if ((l >> 4) == 0) {
#pragma unroll
        for (int i = 0; i < MTW; ++i) {
          const uint32_t r = 16 * (w + 4 * i) + (l & 15);
          if (r < uint32_t(a.twoB)) xs[2 * (rows[r >> 1] + cl) + (r & 1)] = part[i];
        }
      }
      __syncthreads();
    }
    // ---- drain: the tile back to its runs, in batches per thread
    if constexpr (FILL == 1) {
      // 16-byte units; with fill 1 the units at the ends of a run store only their run's amplitude
      constexpr int CH = BF ? 2 : 4;   // the BF16 split's A registers leave room for two in flight
      const uint32_t units = ES >> 1;
      const int32_t last = int32_t(a.BL) - 1;
      auto store_unit = [&](uint32_t ga, int32_t lo0, uint4 v) {
        if (lo0 >= 0 && lo0 < last) {
          st_stream(reinterpret_cast<uint4*>(psi + ga), v);
        } else if (lo0 < 0) {
          st_stream(psi + ga + 1, float2{__uint_as_float(v.z), __uint_as_float(v.w)});
        } else {
          st_stream(psi + ga, float2{__uint_as_float(v.x), __uint_as_float(v.y)});
        }
      };
      uint32_t base = 0;
      for (; base + 256 * CH <= units; base += 256 * CH) {
        uint4 v[CH];
        uint32_t ga[CH];
        int32_t lo0[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          const uint32_t u = base + tid + 256 * j;
          v[j] = *reinterpret_cast<const uint4*>(xs + 4 * u);
          ga[j] = unit_addr(uint32_t(g0), u, &lo0[j]);
        }
        __builtin_amdgcn_sched_barrier(0);   // all LDS reads of the batch are in flight together
#pragma unroll
        for (int j = 0; j < CH; ++j) store_unit(ga[j], lo0[j], v[j]);
      }
      for (uint32_t u = base + tid; u < units; u += 256) {
        int32_t lo0;
        const uint32_t ga = unit_addr(uint32_t(g0), u, &lo0);
        store_unit(ga, lo0, *reinterpret_cast<const uint4*>(xs + 4 * u));
      }
    } else {
      constexpr int CH = 8;
      auto store1 = [&](uint32_t e, float2 v) {
        const uint32_t h = magic_div(e, a.blm);
        st_stream(psi + (g0 + s_hoff[h] + (e - h * a.BL)), v);
      };
      uint32_t base = 0;
      for (; base + 256 * CH <= E; base += 256 * CH) {
        float2 v[CH];
        int64_t ho[CH];
        uint32_t lo[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          const uint32_t e = base + tid + 256 * j, h = magic_div(e, a.blm);
          v[j] = *reinterpret_cast<const float2*>(xs + 2 * e);
          ho[j] = s_hoff[h];
          lo[j] = e - h * a.BL;
        }
        __builtin_amdgcn_sched_barrier(0);   // all LDS reads of the batch are in flight together
#pragma unroll
        for (int j = 0; j < CH; ++j) st_stream(psi + (g0 + ho[j] + lo[j]), v[j]);
      }
      for (uint32_t e = base + tid; e < E; e += 256) store1(e, *reinterpret_cast<const float2*>(xs + 2 * e));
    }
    __syncthreads();
  }
}

// kernel instance names for qd_last_kernel, formatted once per instance as rocprofv3 prints them
template <int MTW, int NTILES, int NH, int KS, bool BF, int WPE, int FILL, bool LEFT>
static const char* rows_label() {
  static thread_local char buf[96] = {0};
  if (!buf[0])
    std::snprintf(buf, sizeof(buf), "k_fused_rows<%d, %d, %d, %d, %s, %d, %d, %s>", MTW, NTILES, NH, KS,
                  BF ? "true" : "false", WPE, FILL, LEFT ? "true" : "false");
  return buf;
}
template <int MTW, int NTILES, int KS, int FILL, bool LEFT, int NBUF>
static const char* pipe_label() {
  static thread_local char buf[96] = {0};
  if (!buf[0])
    std::snprintf(buf, sizeof(buf), "k_fused_pipe<%d, %d, %d, %d, %s, %d>", MTW, NTILES, KS, FILL,
                  LEFT ? "true" : "false", NBUF);
  return buf;
}
template <int MTW, int NTILES, int KS, bool BF>
static const char* general_label() {
  static thread_local char buf[96] = {0};
  if (!buf[0]) std::snprintf(buf, sizeof(buf), "k_fused<%d, %d, %d, %s>", MTW, NTILES, KS, BF ? "true" : "false");
  return buf;
}

static size_t rows_lds(const FusedArgs& a, int ry) {
  return size_t(rows_buf_floats(a.ES)) * sizeof(float) + size_t(2 * ry) * sizeof(int32_t) +
         size_t(a.dH) * sizeof(int64_t);
}

template <int MTW, int NTILES, int NH, int KS, bool BF, int WPE, int FILL, bool LEFT>
static int launch_rows_fill(const FusedArgs& a, hipStream_t st, int per_cu) {
  constexpr int RY = 32 * MTW;
  const size_t lds = rows_lds(a, RY);
  if (lds > kLdsBytes) return fail(QD_EINVAL, "fused tile exceeds the LDS of a CU");
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const unsigned grid = unsigned(std::min<uint64_t>(a.tiles.count, uint64_t(cus) * per_cu));
  auto k = k_fused_rows<MTW, NTILES, NH, KS, BF, WPE, FILL, LEFT>;
  QD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  hipLaunchKernelGGL(k, dim3(grid), dim3(256), lds, st, a);
  QD_HIP(hipGetLastError());
  set_last_kernel(rows_label<MTW, NTILES, NH, KS, BF, WPE, FILL, LEFT>());
  return QD_OK;
}

// one kernel instance per way of moving tiles (each keeps only its own copy code in registers)
template <int MTW, int NTILES, int NH, int KS, bool BF, int WPE>
static int launch_rows(const FusedArgs& a, hipStream_t st, int per_cu) {
  // the single-column path only where the matrix cores bound the kernel (FP32, B <= 81); the BF16
  // kernels are bound by their tile copies, and rebuilding A from its BF16 pair there spills
  if constexpr (NTILES == 6 && !BF && KS == 42) {
    if (a.NT == 16 * (NTILES - 1) + 1) {
      if (a.fill == 0) return launch_rows_fill<MTW, NTILES, NH, KS, BF, WPE, 0, true>(a, st, per_cu);
      if (a.fill == 1) return launch_rows_fill<MTW, NTILES, NH, KS, BF, WPE, 1, true>(a, st, per_cu);
      return launch_rows_fill<MTW, NTILES, NH, KS, BF, WPE, 2, true>(a, st, per_cu);
    }
  }
  if (a.fill == 0) return launch_rows_fill<MTW, NTILES, NH, KS, BF, WPE, 0, false>(a, st, per_cu);
  if (a.fill == 1) return launch_rows_fill<MTW, NTILES, NH, KS, BF, WPE, 1, false>(a, st, per_cu);
  return launch_rows_fill<MTW, NTILES, NH, KS, BF, WPE, 2, false>(a, st, per_cu);
}

// ---------------------------------------------------------------------------------------------
// Double-buffered tiles: one workgroup of 8 waves per CU with two tile buffers in LDS. Waves w and
// w + 4 (one SIMD) hold the same rows of A and take the two halves of the column tiles, so every
// SIMD has two waves of products. Per tile p, every wave
//   issues the loads of tile p + 1 into the other buffer (no wait), runs its products of tile p,
//   waits for its loads (BF16x3: splits the amplitudes it loaded itself), stores its results of
//   tile p from the accumulators straight to HBM, and meets the others at one barrier;
// so the loads of the next tile are in flight during the products, and the stores are issued after
// the wait (the stores of tile p complete while tile p + 1 is worked on; vector memory counters
// would otherwise make the wait for the loads also wait for them).
__host__ __device__ inline uint32_t pipe_in_floats(uint32_t ES) { return (2u * ES + 255u) & ~255u; }

// Tile moves by all 512 threads (thread t: wave t / 64, lane t % 64).
template <int FILL>
__device__ __forceinline__ void pipe_fill_tile(const FusedArgs& a, float2* __restrict__ psi, float* xs, const int64_t* s_hoff,
                                          int64_t g0, uint32_t w, uint32_t l) {
  constexpr uint32_t odd = FILL == 1 ? 1u : 0u;
  if constexpr (FILL == 0 || FILL == 1) {
    const uint32_t units = (FILL == 0 ? a.E : a.ES) >> 1;   // 16 bytes: two adjacent amplitudes
    auto addr = [&](uint32_t u) -> uint32_t {   // global amplitude index of unit u's first amplitude
      if constexpr (FILL == 0) {
        const uint32_t e = 2 * u, h = magic_div(e, a.blm);
        return uint32_t(g0 + s_hoff[h]) + (e - h * a.BL);
      } else {
        const uint32_t h = magic_div(u, a.upm), k = u - h * a.upr;
        const uint32_t start = uint32_t(g0) + uint32_t(s_hoff[h]);
        return start - (start & odd) + 2 * k;
      }
    };
    uint32_t u0 = w * 64;
    for (; u0 + 512 * 3 + 64 <= units; u0 += 512 * 4) {
      uint32_t ga[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) ga[j] = addr(u0 + 512 * j + l);
      __builtin_amdgcn_sched_barrier(0);   // the lookups are in flight together
#pragma unroll
      for (int j = 0; j < 4; ++j) __builtin_amdgcn_global_load_lds(psi + ga[j], xs + 4 * (u0 + 512 * j), 16, 0, kNt);
    }
    for (; u0 < units; u0 += 512) {
      const uint32_t u = u0 + l;
      // lanes past the end read the tile's first unit again (inside the state) into the slack
      const uint32_t ga = addr(u < units ? u : 0u);
      __builtin_amdgcn_global_load_lds(psi + ga, xs + 4 * u0, 16, 0, kNt);
    }
  } else {
    const uint32_t units = a.E * 2;   // 4 bytes: one part of one amplitude
    const float* pf = reinterpret_cast<const float*>(psi);
    auto addr = [&](uint32_t f) -> uint64_t {
      const uint32_t e = f >> 1, h = magic_div(e, a.blm);
      return 2 * uint64_t(g0 + s_hoff[h] + (e - h * a.BL)) + (f & 1u);
    };
    uint32_t u0 = w * 64;
    for (; u0 + 512 * 3 + 64 <= units; u0 += 512 * 4) {
      uint64_t ga[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) ga[j] = addr(u0 + 512 * j + l);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < 4; ++j) __builtin_amdgcn_global_load_lds(pf + ga[j], xs + u0 + 512 * j, 4, 0, kNt);
    }
    for (; u0 < units; u0 += 512) {
      const uint32_t f = u0 + l;
      const uint64_t ga = addr(f < units ? f : 0u);
      __builtin_amdgcn_global_load_lds(pf + ga, xs + u0, 4, 0, kNt);
    }
  }
}

// Fill 0 and 1: each lane's 16-byte units (u = 64 w + l + 512 m) as offsets from the tile origin,
// computed once per launch, so that loading a tile takes two integer operations per unit instead of
// a division and a table lookup. Unit u of a fill-1 tile starts at origin + rel - parity, where the
// parity (origin + run offset) & 1 is the origin's parity xor the run offset's (bit m of par).
constexpr int kPipeUnits = 8;   // units per lane: 512 lanes x 8 units x 2 amplitudes cover every tile
struct PipeUnits {
  uint32_t rel[kPipeUnits];
  uint32_t par;
};

template <int FILL>
__device__ __forceinline__ void pipe_units_init(const FusedArgs& a, PipeUnits& pu, uint32_t w, uint32_t l) {
  static_assert(FILL == 0 || FILL == 1, "16-byte units");
  const uint32_t units = (FILL == 0 ? a.E : a.ES) >> 1;
  pu.par = 0;
#pragma unroll
  for (int m = 0; m < kPipeUnits; ++m) {
    const uint32_t u = w * 64 + l + 512u * m;
    uint32_t rel = 0, par = 0;   // lanes past the end: the tile's first unit (read into the slack)
    if (u < units) {
      if constexpr (FILL == 0) {
        const uint32_t e = 2 * u, h = magic_div(e, a.blm);
        rel = uint32_t(a.hoff[h]) + (e - h * a.BL);
      } else {
        const uint32_t h = magic_div(u, a.upm), k = u - h * a.upr;
        rel = uint32_t(a.hoff[h]) + 2 * k;
        par = uint32_t(a.hoff[h]) & 1u;
      }
    }
    pu.rel[m] = rel;
    pu.par |= par << m;
  }
}

template <int FILL>
__device__ __forceinline__ void pipe_load_units(const FusedArgs& a, float2* __restrict__ psi, float* xs,
                                                const PipeUnits& pu, uint32_t g0, uint32_t w) {
  const uint32_t units = (FILL == 0 ? a.E : a.ES) >> 1;
#pragma unroll
  for (int m = 0; m < kPipeUnits; ++m) {
    const uint32_t u0 = w * 64 + 512u * m;
    if (u0 < units) {
      uint32_t ga = g0 + pu.rel[m];
      if constexpr (FILL == 1) ga -= (g0 ^ (pu.par >> m)) & 1u;
      __builtin_amdgcn_global_load_lds(psi + ga, xs + 4 * u0, 16, 0, kNt);
    }
  }
}

// The products of one wave over one tile: its MTW row tiles of A times its NTH column tiles of X,
// except the (row tile i, column tile t) pairs whose bit t MTW + i is set in SKIPM. `between` runs
// after the first operands are read and before the products (the next tile's loads: issued after
// those reads, they make no read of this tile wait for them).
template <int MTW, uint32_t SKIPM>
__host__ __device__ constexpr bool pp_on(int i, int t) { return ((SKIPM >> (t * MTW + i)) & 1u) == 0; }
template <int MTW, uint32_t SKIPM>
__host__ __device__ constexpr bool pp_tile(int t) {
  bool any = false;
  for (int i = 0; i < MTW; ++i) any = any || pp_on<MTW, SKIPM>(i, t);
  return any;
}

template <int MTW, int NTH, int KS, uint32_t SKIPM, typename F>
__device__ __forceinline__ void pipe_products(v4f (&acc)[MTW][NTH], const float* xs, const int32_t* rows,
                                              const int32_t (&cp)[NTH], const float (&af)[MTW][KS], uint32_t l,
                                              F&& between) {
#pragma unroll
  for (int i = 0; i < MTW; ++i)
#pragma unroll
    for (int t = 0; t < NTH; ++t) acc[i][t] = v4f{0.f, 0.f, 0.f, 0.f};
  // K in pairs of steps: in steps 2 j and 2 j + 1 lane l takes the real and the imaginary part
  // of amplitude (row y = 4 j + (l >> 4), column n = 16 nt + (l & 15)), one 8-byte LDS read for
  // two products. The operands of pair j + 1 are loaded before the products of pair j. An odd KS
  // ends with one single step over real rows k = 4 (KS - 1) + (l >> 4): complex row
  // 2 (KS - 1) + (l >> 5), part (l >> 4) & 1.
  constexpr int KP = KS / 2;
  constexpr bool ODD = (KS & 1) != 0;
  constexpr int NL = KP + (ODD ? 1 : 0);   // operand loads: the pairs, then the single step
  const float2* x2 = reinterpret_cast<const float2*>(xs);
  const int32_t* rpl = rows + (l >> 4);
  // row of load j (a pair: 4 j + (l >> 4); the single step: 2 (KS - 1) + (l >> 5))
  auto lrow = [&](int j) -> int32_t { return (ODD && j == KP) ? rows[2 * (KS - 1) + int(l >> 5)] : rpl[4 * j]; };
  float2 b[2][NTH];
  int32_t rk = lrow(0);
#pragma unroll
  for (int t = 0; t < NTH; ++t)
    if (pp_tile<MTW, SKIPM>(t)) b[0][t] = x2[rk + cp[t]];
  if (NL > 1) rk = lrow(1);
  between();
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    if (j + 1 < NL) {
#pragma unroll
      for (int t = 0; t < NTH; ++t)
        if (pp_tile<MTW, SKIPM>(t)) b[(j + 1) & 1][t] = x2[rk + cp[t]];
      if (j + 2 < NL) rk = lrow(j + 2);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (!(ODD && j == KP)) {
#pragma unroll
      for (int t = 0; t < NTH; ++t)
#pragma unroll
        for (int i = 0; i < MTW; ++i)
          if (pp_on<MTW, SKIPM>(i, t)) {
            acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][2 * j], b[j & 1][t].x, acc[i][t], 0, 0, 0);
            acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][2 * j + 1], b[j & 1][t].y, acc[i][t], 0, 0, 0);
          }
    } else {
      const bool im = ((l >> 4) & 1u) != 0;   // this lane's part of the amplitude
#pragma unroll
      for (int t = 0; t < NTH; ++t) {
        const float2 v = b[j & 1][t];   // (selecting from a copy keeps b in registers)
        const float bv = im ? v.y : v.x;
#pragma unroll
        for (int i = 0; i < MTW; ++i)
          if (pp_on<MTW, SKIPM>(i, t))
            acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][KS - 1], bv, acc[i][t], 0, 0, 0);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Column tiles of the two waves of a SIMD (wave half hf = w / 4). Without the single column:
// NTILES / 2 each. With it (81 columns: tiles 0-4 on the matrix cores, tile 5 = column 80 on the
// vector units), balanced as 8 and 7 products per K step: half 0 takes tiles 0, 1 and the first
// two row tiles of tile 2; half 1 the last row tile of tile 2, tiles 3, 4 and the single column.
template <int MTW, int NTILES, bool LEFT>
struct PipeSplit {
  static constexpr bool BAL = LEFT && MTW == 3 && NTILES == 6;
  static constexpr int NT0 = BAL ? 3 : NTILES / 2, NT1 = BAL ? 4 : NTILES / 2;
  static constexpr int CB1 = BAL ? 2 : NTILES / 2;   // first column tile of half 1
  static constexpr uint32_t M0 = BAL ? (1u << (2 * MTW + 2)) : 0u;
  static constexpr uint32_t M1 = BAL ? ((1u << 0) | (1u << 1) | (((1u << MTW) - 1u) << (3 * MTW)))
                                     : (LEFT ? (((1u << MTW) - 1u) << ((NT1 - 1) * MTW)) : 0u);
  static constexpr int NTMAX = NT0 > NT1 ? NT0 : NT1;
};

// One tile of the double-buffered kernel (tile p from xs, tile p + 1 into xn) for wave half H. The
// restrict qualifiers tell the compiler the two buffers are distinct, so it does not wait for the
// loads into xn before the products read xs (the loads are issued after the first operand reads).
template <int MTW, int NTILES, int KS, int FILL, bool LEFT, int H>
__device__ __forceinline__ void pipe_phase(const FusedArgs& a, float* __restrict__ xs, float* __restrict__ xn,
                                           uint32_t p, uint32_t ntile, const int64_t* s_hoff,
                                           const int32_t* s_rowpos, const uint32_t* s_wrow,
                                           const int32_t (&cpa)[PipeSplit<MTW, NTILES, LEFT>::NTMAX],
                                           const float (&af)[MTW][KS], int32_t cl, const PipeUnits& pu,
                                           uint32_t w, uint32_t l) {
  using S = PipeSplit<MTW, NTILES, LEFT>;
  constexpr int RY = 32 * MTW;
  constexpr int NTH = H ? S::NT1 : S::NT0;
  constexpr uint32_t M = H ? S::M1 : S::M0;
  constexpr int CB = H ? S::CB1 : 0;
  constexpr bool LC = LEFT && H == 1;   // this half computes the single column
  float2* __restrict__ psi = a.psi;
  const uint32_t q = w & 3u;
  const uint32_t g0 = uint32_t(fm_offset(a.tiles, blockIdx.x + p * gridDim.x));
  const int32_t* rows = s_rowpos + (FILL == 1 ? RY * int32_t(g0 & 1u) : 0);
  int32_t cp[NTH];
#pragma unroll
  for (int t = 0; t < NTH; ++t) cp[t] = cpa[t];

  v4f acc[MTW][NTH];
  pipe_products<MTW, NTH, KS, M>(acc, xs, rows, cp, af, l, [&] {
    if (p + 1 < ntile) {
      const int64_t gn = fm_offset(a.tiles, blockIdx.x + (p + 1) * gridDim.x);
      if constexpr (FILL == 2) pipe_fill_tile<FILL>(a, psi, xn, s_hoff, gn, w, l);
      else pipe_load_units<FILL>(a, psi, xn, pu, uint32_t(gn), w);
    }
  });
  float part[MTW];
  if constexpr (LC) {
    // the single column on the vector units: lane (row 16 (q + 4 i) + (l & 15)) sums A[r][k] x[k]
    // over its own k, then the four lanes of the row by wavefront shuffles
    const float2* x2 = reinterpret_cast<const float2*>(xs);
#pragma unroll
    for (int i = 0; i < MTW; ++i) part[i] = 0.f;
#pragma unroll
    for (int j = 0; j < KS / 2; ++j) {   // complex row 4 j + (l >> 4): real rows 2 (4 j + (l >> 4)) + c
      const float2 x = x2[rows[4 * j + int(l >> 4)] + cl];
#pragma unroll
      for (int i = 0; i < MTW; ++i) part[i] = fmaf(af[i][2 * j + 1], x.y, fmaf(af[i][2 * j], x.x, part[i]));
    }
    if constexpr ((KS & 1) != 0) {   // the single last step: complex row 2 (KS - 1) + (l >> 5)
      const float2 x = x2[rows[2 * (KS - 1) + int(l >> 5)] + cl];
      const float xv = ((l >> 4) & 1u) ? x.y : x.x;
#pragma unroll
      for (int i = 0; i < MTW; ++i) part[i] = fmaf(af[i][KS - 1], xv, part[i]);
    }
#pragma unroll
    for (int i = 0; i < MTW; ++i) {
      part[i] += __shfl_xor(part[i], 16);
      part[i] += __shfl_xor(part[i], 32);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);   // this lane's loads of tile p + 1 (and the stores of tile p - 1)
  // results of tile p from the accumulators to HBM: amplitude (y, n) at g0 + wrow[y] + colpos[n]
  const uint32_t yend = uint32_t(a.twoB / 2);
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
    const uint32_t y0 = 8 * (q + 4 * i) + 2 * (l >> 4);   // result rows 2 y0 .. 2 y0 + 3
    const uint32_t o0 = g0 + s_wrow[y0], o1 = g0 + s_wrow[y0 + 1];
#pragma unroll
    for (int t = 0; t < NTH; ++t) {
      const uint32_t n = 16 * (CB + t) + (l & 15);
      if (pp_on<MTW, M>(i, t) && n < a.NT) {
        if (y0 < yend) psi[o0 + uint32_t(cp[t])] = float2{acc[i][t][0], acc[i][t][1]};
        if (y0 + 1 < yend) psi[o1 + uint32_t(cp[t])] = float2{acc[i][t][2], acc[i][t][3]};
      }
    }
  }
  if constexpr (LC) {
    if ((l >> 4) == 0) {
      float* pf = reinterpret_cast<float*>(psi);
#pragma unroll
      for (int i = 0; i < MTW; ++i) {
        const uint32_t r = 16 * (q + 4 * i) + (l & 15);
        if (r < uint32_t(a.twoB)) pf[2 * uint64_t(g0 + s_wrow[r >> 1] + uint32_t(cl)) + (r & 1)] = part[i];
      }
    }
  }
}

template <int MTW, int NTILES, int KS, int FILL, bool LEFT, int NBUF>
__global__ __launch_bounds__(512, 1) void k_fused_pipe(FusedArgs a) {
  using S = PipeSplit<MTW, NTILES, LEFT>;
  constexpr int KPAD = 64 * MTW;
  constexpr int RY = KPAD / 2;
  static_assert(NTILES % 2 == 0, "column tiles split between the two waves of a SIMD");
  __shared__ __align__(16) float xbuf[2][NBUF];
  __shared__ int32_t s_rowpos[2 * RY];
  __shared__ uint32_t s_wrow[RY];
  extern __shared__ __align__(16) unsigned char lds_raw[];
  int64_t* s_hoff = reinterpret_cast<int64_t*>(lds_raw);
  // wave index through readfirstlane: the compiler sees it uniform, so the per-half branch is
  // scalar (a wave runs one set of products, not both under an execution mask)
  const uint32_t tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
  const uint32_t q = w & 3u;          // row tiles q + 4 i
  const uint32_t hf = w >> 2;
  const uint32_t nrow = FILL == 1 ? 2u * RY : uint32_t(RY);
  for (uint32_t h = tid; h < a.dH; h += 512) s_hoff[h] = a.hoff[h];
  for (uint32_t y = tid; y < nrow; y += 512) s_rowpos[y] = a.rowpos[y];
  for (uint32_t y = tid; y < uint32_t(RY); y += 512) s_wrow[y] = a.wrow[y];
  // LDS tile position of this lane's column in each of its column tiles = its offset in a run
  int32_t cp[S::NTMAX];
  {
    const int cb = hf ? S::CB1 : 0;
#pragma unroll
    for (int t = 0; t < S::NTMAX; ++t) cp[t] = a.colpos[16 * std::min(cb + t, NTILES - 1) + (l & 15)];
  }
  const int32_t cl = a.colpos[16 * (NTILES - 1)];   // the single column (LEFT)
  float af[MTW][KS];
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
    const int row = 16 * (int(q) + 4 * i) + int(l & 15);
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      // step kk = 2 j + c of a pair: real row k = 2 (4 j + (l >> 4)) + c; an odd last step: 4 kk + (l >> 4)
      const int k = ((KS & 1) && kk == KS - 1) ? 4 * kk + int(l >> 4) : 2 * (4 * (kk >> 1) + int(l >> 4)) + (kk & 1);
      af[i][kk] = a.a32[size_t(row) * KPAD + k];
    }
  }
  PipeUnits pu;
  if constexpr (FILL != 2) pipe_units_init<FILL>(a, pu, w, l);
  const uint32_t ntile = blockIdx.x < a.tiles.count ? (a.tiles.count - 1 - blockIdx.x) / gridDim.x + 1 : 0u;
  __syncthreads();   // tables in LDS
  if (ntile > 0) {
    const int64_t g0 = fm_offset(a.tiles, blockIdx.x);
    if constexpr (FILL == 2) pipe_fill_tile<FILL>(a, a.psi, xbuf[0], s_hoff, g0, w, l);
    else pipe_load_units<FILL>(a, a.psi, xbuf[0], pu, uint32_t(g0), w);
  }
  // tile 0 and the rows of A have arrived (waiting here on every path also tells the compiler that
  // no load of A is still pending inside the loop)
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();   // tile 0 in LDS
  for (uint32_t p = 0; p < ntile; ++p) {
    if (hf)
      pipe_phase<MTW, NTILES, KS, FILL, LEFT, 1>(a, xbuf[p & 1u], xbuf[(p + 1) & 1u], p, ntile, s_hoff, s_rowpos,
                                                 s_wrow, cp, af, cl, pu, w, l);
    else
      pipe_phase<MTW, NTILES, KS, FILL, LEFT, 0>(a, xbuf[p & 1u], xbuf[(p + 1) & 1u], p, ntile, s_hoff, s_rowpos,
                                                 s_wrow, cp, af, cl, pu, w, l);
    __syncthreads();   // every wave has read its operands of tile p; tile p + 1 is in LDS
  }
}

// whether a block's tile buffers fit a kernel instance with NBUF floats per buffer
template <int MTW, int NBUF>
static bool pipe_fits(const FusedArgs& a) {
  const size_t lds = size_t(2) * NBUF * sizeof(float) + size_t(96 * MTW) * sizeof(int32_t) + size_t(a.dH) * sizeof(int64_t);
  const bool units_fit = a.fill == 2 || ((a.fill == 0 ? a.E : a.ES) >> 1) <= 512u * kPipeUnits;
  return pipe_in_floats(a.ES) <= uint32_t(NBUF) && lds <= kLdsBytes && units_fit;
}

template <int MTW, int NTILES, int KS, int NBUF, int FILL, bool LEFT>
static int launch_pipe_fill(const FusedArgs& a, hipStream_t st) {
  const size_t dyn = size_t(a.dH) * sizeof(int64_t);
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const unsigned grid = unsigned(std::min<uint64_t>(a.tiles.count, uint64_t(cus)));
  auto k = k_fused_pipe<MTW, NTILES, KS, FILL, LEFT, NBUF>;
  QD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, int(dyn)));
  hipLaunchKernelGGL(k, dim3(grid), dim3(512), dyn, st, a);
  QD_HIP(hipGetLastError());
  set_last_kernel(pipe_label<MTW, NTILES, KS, FILL, LEFT, NBUF>());
  return QD_OK;
}

template <int MTW, int NTILES, int KS, int NBUF>
static int launch_pipe(const FusedArgs& a, hipStream_t st) {
  if constexpr (NTILES == 6 && KS == 41) {
    if (a.NT == 16 * (NTILES - 1) + 1) {
      if (a.fill == 0) return launch_pipe_fill<MTW, NTILES, KS, NBUF, 0, true>(a, st);
      if (a.fill == 1) return launch_pipe_fill<MTW, NTILES, KS, NBUF, 1, true>(a, st);
      return launch_pipe_fill<MTW, NTILES, KS, NBUF, 2, true>(a, st);
    }
  }
  if (a.fill == 0) return launch_pipe_fill<MTW, NTILES, KS, NBUF, 0, false>(a, st);
  if (a.fill == 1) return launch_pipe_fill<MTW, NTILES, KS, NBUF, 1, false>(a, st);
  return launch_pipe_fill<MTW, NTILES, KS, NBUF, 2, false>(a, st);
}

template <int MTW, int NTILES, int KS, bool BF>
static int launch_one(const FusedArgs& a, hipStream_t st, int per_cu) {
  constexpr int P = 64 * MTW + 4;
  const size_t lds = size_t(NTILES) * 16 * P * sizeof(float) + size_t(a.dH) * (sizeof(int64_t) + sizeof(int32_t));
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const unsigned grid = unsigned(std::min<uint64_t>(a.tiles.count, uint64_t(cus) * per_cu));
  auto k = k_fused<MTW, NTILES, KS, BF>;
  QD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  hipLaunchKernelGGL(k, dim3(grid), dim3(256), lds, st, a);
  QD_HIP(hipGetLastError());
  set_last_kernel(general_label<MTW, NTILES, KS, BF>());
  return QD_OK;
}

// Kernel shapes by block dimension B (2B real rows): KPAD = 64 MTW >= 2B.
//   B <= 32: 1 tile of A per wave; B <= 64: 2; B <= 81: 3 (41 FP32 K steps); B <= 96: 3; B <= 128: 4.
// Persistent workgroups per CU: as many as registers and LDS hold (4 for B <= 32, 3 for B <= 64, 2
// above), so that one workgroup's tile copies overlap the others' products; double-buffering the
// tile in one workgroup measured slower on the 64-wide blocks (it leaves room for two).
static int variant_of(int B) { return B <= 32 ? 0 : (B <= 64 ? 1 : (B <= 81 ? 2 : (B <= 96 ? 3 : 4))); }
static int variant_kpad(int v) { return v == 0 ? 64 : (v == 1 ? 128 : (v <= 3 ? 192 : 256)); }
static int variant_ntiles(int v) { return (v == 2 || v == 3) ? 6 : 4; }

int launch_fused_block(qd_state* s, const qd_fused* f, int b, int mode) {
  const FusedBlockDev& d = f->dev[b];
  if (!d.geom_ok) return fail(QD_EINVAL, "fused block has no matrix-core tiling");
  FusedArgs a = d.args;
  a.psi = reinterpret_cast<float2*>(s->data);
  if (a.tiles.count == 0) return QD_OK;
  // the spare amplitude of an odd run may be the one after the last: read only inside the buffer
  if (a.fill == 1 && (uint64_t(s->cap_bytes) < (uint64_t(s->reg.D) + 1) * 8u ||
                      (reinterpret_cast<uintptr_t>(s->data) & 15u) != 0)) {
    a.fill = 2;
    a.ES = a.E;
    a.rowpos = d.variant <= 3 ? d.tab_rowpos : nullptr;
  }
  const bool bf = mode == QD_MODE_BF16X3_MFMA;
  // FP32 blocks of 64 < B <= 81: the double-buffered kernel where its two tile buffers (each as
  // large as the largest fill-1 tile of an 81-wide block over qutrits) fit the LDS of a CU. For
  // B <= 64 several workgroups per CU of the kernel below measured faster; for B > 81 the
  // double-buffered kernel's registers spill.
  if (!bf && a.rowpos && a.NT <= uint32_t(16 * variant_ntiles(d.variant))) {
    switch (d.variant) {
      case 2: if (pipe_fits<3, 13312>(a)) return launch_pipe<3, 6, 41, 13312>(a, s->stream); break;
      default: break;
    }
  }
  if (a.rowpos && a.NT <= uint32_t(16 * variant_ntiles(d.variant))) {
    switch (d.variant) {
      case 0: return bf ? launch_rows<1, 4, 1, 2, true, 2>(a, s->stream, 4)
                        : launch_rows<1, 4, 1, 16, false, 2>(a, s->stream, 4);
      case 1: return bf ? launch_rows<2, 4, 1, 4, true, 2>(a, s->stream, 3)
                        : launch_rows<2, 4, 1, 32, false, 2>(a, s->stream, 3);
      case 2: return bf ? launch_rows<3, 6, 2, 6, true, 2>(a, s->stream, 2)
                        : launch_rows<3, 6, 2, 42, false, 2>(a, s->stream, 2);
      case 3: return bf ? launch_rows<3, 6, 2, 6, true, 2>(a, s->stream, 2)
                        : launch_rows<3, 6, 2, 48, false, 2>(a, s->stream, 2);
      default: break;  // B > 96 keeps the general kernel
    }
  }
  switch (d.variant) {
    case 0: return bf ? launch_one<1, 4, 2, true>(a, s->stream, 3) : launch_one<1, 4, 16, false>(a, s->stream, 3);
    case 1: return bf ? launch_one<2, 4, 4, true>(a, s->stream, 2) : launch_one<2, 4, 32, false>(a, s->stream, 2);
    case 2: return bf ? launch_one<3, 6, 6, true>(a, s->stream, 2) : launch_one<3, 6, 41, false>(a, s->stream, 2);
    case 3: return bf ? launch_one<3, 6, 6, true>(a, s->stream, 2) : launch_one<3, 6, 48, false>(a, s->stream, 2);
    default: return bf ? launch_one<4, 4, 8, true>(a, s->stream, 1) : launch_one<4, 4, 64, false>(a, s->stream, 1);
  }
}

int fused_kpad(int B) { return variant_kpad(variant_of(B)); }

// Tile geometry of a block on its register: the low suffix L = {pq..n-1} grows from the least
// significant qudit while the non-window part of L (the columns of a tile) stays within ntmax.
int fused_geometry(const Register& r, FusedBlockDev* d) {
  const FusedBlockInfo& in = d->info;
  const int B = in.B;
  d->variant = variant_of(B);
  const int ntiles = variant_ntiles(d->variant);
  const uint32_t ntmax = 16u * ntiles;
  bool inwin[QD_MAX_QUDITS] = {};
  for (int j = 0; j < in.k; ++j) inwin[in.window[j]] = true;
  int pq = r.n;
  uint64_t BL = 1, NT = 1;
  while (pq > 0) {
    const int q = pq - 1;
    const uint64_t nNT = inwin[q] ? NT : NT * r.dims[q];
    if (nNT > ntmax) break;
    pq = q;
    BL *= r.dims[q];
    NT = nNT;
  }
  uint64_t dH = 1;
  for (int q = 0; q < pq; ++q)
    if (inwin[q]) dH *= r.dims[q];
  FusedArgs& a = d->args;
  std::memset(&a, 0, sizeof(a));
  a.Kp = d->Kp;
  a.twoB = 2 * B;
  a.BL = uint32_t(BL);
  a.dH = uint32_t(dH);
  a.E = uint32_t(BL * dH);
  a.NT = uint32_t(NT);
  a.blm = make_magic32(uint32_t(BL));
  a.high_window = 1;
  for (int q = pq; q < r.n; ++q)
    if (inwin[q]) a.high_window = 0;
  // tile origins: digits of the non-window qudits above L
  int role[QD_MAX_QUDITS] = {};
  for (int q = 0; q < r.n; ++q) role[q] = inwin[q] ? 1 : 0;
  int rc = fill_slicemap(make_groups(r, role, nullptr, 0, pq), 0, &a.tiles);
  if (rc) return rc;
  // window-local index weights: window qudit j (ascending) has weight prod of later window dims
  int64_t wmul[QD_MAX_QUDITS] = {};
  {
    int64_t m = 1;
    for (int j = in.k - 1; j >= 0; --j) {
      wmul[in.window[j]] = m;
      m *= r.dims[in.window[j]];
    }
  }
  // runs: h over the window qudits above L (mixed radix, ascending qudit most significant)
  std::vector<int64_t> hoff(dH);
  std::vector<int32_t> yh(dH);
  for (uint64_t h = 0; h < dH; ++h) {
    uint64_t rem = h;
    int64_t off = 0, y = 0;
    for (int q = pq - 1; q >= 0; --q)
      if (inwin[q]) {
        const uint64_t dg = rem % r.dims[q];
        rem /= r.dims[q];
        off += int64_t(dg) * r.strides[q];
        y += int64_t(dg) * wmul[q];
      }
    hoff[h] = off;
    yh[h] = int32_t(y);
  }
  // inside a run: amplitude lo -> (column n, window-local part of y)
  std::vector<uint32_t> lmap(BL);
  for (uint64_t lo = 0; lo < BL; ++lo) {
    uint64_t rem = lo;
    uint64_t n = 0, nmul = 1, y = 0;
    for (int q = r.n - 1; q >= pq; --q) {
      const uint64_t dg = rem % r.dims[q];
      rem /= r.dims[q];
      if (inwin[q]) {
        y += dg * uint64_t(wmul[q]);
      } else {
        n += dg * nmul;
        nmul *= r.dims[q];
      }
    }
    lmap[lo] = uint32_t(n << 16) | uint32_t(y);
  }
  // position of amplitude (y, n) inside a tile in HBM order: rowpos[y] + colpos[n]
  const int RY = variant_kpad(d->variant) / 2;
  const int NC = 16 * ntiles;
  std::vector<int32_t> rowpos(RY, 0), colpos(NC, 0);   // padding rows and columns alias the first
  std::vector<uint32_t> wrow(RY, 0);
  {
    // offset inside the run of each window-local digit combination that lies in L, and of each column
    std::vector<int64_t> y_lo(size_t(B), 0);
    for (uint64_t lo = 0; lo < BL; ++lo) {
      const uint32_t lm = lmap[lo];
      const uint32_t n = lm >> 16, yl = lm & 0xFFFFu;
      if (n == 0) y_lo[yl] = int64_t(lo);
      if (yl == 0 && n < uint32_t(NC)) colpos[n] = int32_t(lo);
    }
    // y = yh[h] + yl with yl ranging over the window digits inside L: enumerate both
    std::vector<int32_t> yl_list;
    for (uint64_t lo = 0; lo < BL; ++lo)
      if ((lmap[lo] >> 16) == 0) yl_list.push_back(int32_t(lmap[lo] & 0xFFFFu));
    for (uint64_t h = 0; h < dH; ++h)
      for (int32_t yl : yl_list) {
        const int y = yh[h] + yl;
        if (y < RY) {
          rowpos[y] = int32_t(h * BL + uint64_t(y_lo[yl]));
          wrow[y] = uint32_t(hoff[h] + y_lo[yl]);
        }
      }
  }
  QD_HIP(hipMalloc((void**)&d->tab_rowpos, sizeof(int32_t) * RY));
  QD_HIP(hipMalloc((void**)&d->tab_colpos, sizeof(int32_t) * NC));
  QD_HIP(hipMemcpy(d->tab_rowpos, rowpos.data(), sizeof(int32_t) * RY, hipMemcpyHostToDevice));
  QD_HIP(hipMemcpy(d->tab_colpos, colpos.data(), sizeof(int32_t) * NC, hipMemcpyHostToDevice));
  QD_HIP(hipMalloc((void**)&d->tab_wrow, sizeof(uint32_t) * RY));
  QD_HIP(hipMemcpy(d->tab_wrow, wrow.data(), sizeof(uint32_t) * RY, hipMemcpyHostToDevice));
  a.wrow = d->tab_wrow;
  a.rowpos = d->variant <= 3 ? d->tab_rowpos : nullptr;
  a.colpos = d->tab_colpos;
  // tile moves in 16-byte units: an odd run length keeps BL + 1 LDS slots per run, the run starting
  // at slot (tile origin + run offset) & 1, so the row table depends on the origin's parity
  if ((BL & 1u) == 0) {
    a.fill = 0;
    a.upr = uint32_t(BL / 2);
    a.ES = a.E;
  } else {
    a.fill = 1;
    a.upr = uint32_t((BL + 1) / 2);
    a.ES = uint32_t(dH * (BL + 1));
    std::vector<int32_t> rp2(2 * size_t(RY), 0);
    for (int par = 0; par < 2; ++par)
      for (int y = 0; y < RY; ++y) {
        const int32_t pos = rowpos[y];                 // h BL + offset inside the run
        const uint64_t h = uint64_t(pos) / BL, lo = uint64_t(pos) % BL;
        const int32_t shift = int32_t((uint64_t(par) + uint64_t(hoff[h])) & 1u);
        rp2[size_t(par) * RY + y] = int32_t(h * (BL + 1) + lo) + shift;
      }
    QD_HIP(hipMalloc((void**)&d->tab_rowpos_odd, sizeof(int32_t) * 2 * RY));
    QD_HIP(hipMemcpy(d->tab_rowpos_odd, rp2.data(), sizeof(int32_t) * 2 * RY, hipMemcpyHostToDevice));
    if (d->variant <= 3) a.rowpos = d->tab_rowpos_odd;
  }
  a.upm = make_magic32(a.upr);
  QD_HIP(hipMalloc((void**)&d->tab_hoff, sizeof(int64_t) * dH));
  QD_HIP(hipMalloc((void**)&d->tab_yh, sizeof(int32_t) * dH));
  QD_HIP(hipMalloc((void**)&d->tab_lmap, sizeof(uint32_t) * BL));
  QD_HIP(hipMemcpy(d->tab_hoff, hoff.data(), sizeof(int64_t) * dH, hipMemcpyHostToDevice));
  QD_HIP(hipMemcpy(d->tab_yh, yh.data(), sizeof(int32_t) * dH, hipMemcpyHostToDevice));
  QD_HIP(hipMemcpy(d->tab_lmap, lmap.data(), sizeof(uint32_t) * BL, hipMemcpyHostToDevice));
  a.hoff = d->tab_hoff;
  a.yh = d->tab_yh;
  a.lmap = d->tab_lmap;
  a.a32 = d->a32;
  a.ahi = reinterpret_cast<const __bf16*>(d->ahi);
  a.alo = reinterpret_cast<const __bf16*>(d->alo);
  d->geom_ok = true;
  return QD_OK;
}

}  // namespace qd
