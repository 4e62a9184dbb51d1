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
#include <cstring>

#include "qd_fused.h"

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

// Moves the E amplitudes of a tile between HBM and the LDS column layout. TO_LDS: HBM -> LDS.
template <bool TO_LDS>
__device__ __forceinline__ void tile_move(const FusedArgs& a, float2* __restrict__ psi, float* xs, uint32_t P,
                                          const int64_t* s_hoff, const int32_t* s_yh, int64_t g0) {
  constexpr int CH = 8;  // amplitudes in flight per thread
  const uint32_t tid = threadIdx.x;
  for (uint32_t base = 0; base < a.E; base += 256 * CH) {
    float vr[CH], vi[CH];
    uint32_t pos[CH];
    int64_t goff[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const uint32_t idx = base + tid + 256 * j;
      pos[j] = 0xFFFFFFFFu;
      if (idx < a.E) {
        const uint32_t h = magic_div(idx, a.blm);
        const uint32_t lo = idx - h * a.BL;
        const uint32_t lm = a.lmap[lo];
        const uint32_t n = lm >> 16, y = uint32_t(s_yh[h]) + (lm & 0xFFFFu);
        pos[j] = n * P + 2 * y;
        goff[j] = g0 + s_hoff[h] + lo;
        if (TO_LDS) {
          const float2 t = psi[goff[j]];
          vr[j] = t.x;
          vi[j] = t.y;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      if (pos[j] != 0xFFFFFFFFu) {
        float2* p2 = reinterpret_cast<float2*>(xs + pos[j]);
        if (TO_LDS) {
          float2 t;
          t.x = vr[j];
          t.y = vi[j];
          *p2 = t;
        } else {
          const float2 t = *p2;
          vr[j] = t.x;
          vi[j] = t.y;
        }
      }
    }
    if (!TO_LDS) {
#pragma unroll
      for (int j = 0; j < CH; ++j)
        if (pos[j] != 0xFFFFFFFFu) {
          float2 t;
          t.x = vr[j];
          t.y = vi[j];
          psi[goff[j]] = t;
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
    tile_move<true>(a, psi, xs, P, s_hoff, s_yh, g0);
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
    tile_move<false>(a, psi, xs, P, s_hoff, s_yh, g0);
    __syncthreads();
  }
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
  return QD_OK;
}

// Kernel shapes by block dimension B (2B real rows): KPAD = 64 MTW >= 2B.
//   B <= 32: 1 tile of A per wave; B <= 64: 2; B <= 81: 3 (41 FP32 K steps); B <= 96: 3; B <= 128: 4.
static int variant_of(int B) { return B <= 32 ? 0 : (B <= 64 ? 1 : (B <= 81 ? 2 : (B <= 96 ? 3 : 4))); }
static int variant_kpad(int v) { return v == 0 ? 64 : (v == 1 ? 128 : (v <= 3 ? 192 : 256)); }
static int variant_ntiles(int v) { return (v == 2 || v == 3) ? 6 : 4; }

int launch_fused_block(qd_state* s, const qd_fused* f, int b, int mode) {
  const FusedBlockDev& d = f->dev[b];
  if (!d.geom_ok) return fail(QD_EINVAL, "fused block has no matrix-core tiling");
  FusedArgs a = d.args;
  a.psi = reinterpret_cast<float2*>(s->data);
  if (a.tiles.count == 0) return QD_OK;
  const bool bf = mode == QD_MODE_BF16X3_MFMA;
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
