// Gate-application kernels for gfx950 and their launcher.
//
// One generalized gate (Sec. 2.1) applied in place: every slice of the register (the d_T
// amplitudes that share all non-target digits) whose control digits match is multiplied by U.
// That is the Kronecker-embedded Moment operator I (x) U (x) I of Sec. 3.5 applied to the state
// vector, at O(D d_T) cost.
//
// Kernel families (each HBM-bound: at most 8 d_T flops per 2 x 16 bytes moved):
//   k_slices_direct  one slice per thread. Used when every target has a stride >= run_min (or at
//                    least one line, for controls inside a line that leave lines inactive), so the
//                    lanes of a wavefront take consecutive low digits and each load instruction
//                    reads one contiguous run.
//   k_slices_tiled   a low-stride target: the workgroup stages a tile of whole slices in LDS with
//                    contiguous coalesced loads (runs of the low suffix of the register), mixes
//                    each slice inside LDS and writes the tile back coalesced.
//   k_diag           diagonal gates (Z_d, controlled phases): elementwise, consecutive lanes on
//                    consecutive amplitudes whatever the target strides.
//   k_dense_generic  any d_T <= 1024 and any register size (64-bit indices): slices gathered into
//                    LDS, U read from device memory.
// The slice kernels take U (dense) or a destination/phase table (monomial: X_{+a}, controlled
// shifts, qudit swaps) inside the kernel arguments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "qd_internal.h"
#include "qd_stream.h"

namespace qd {

template <typename R> struct CxT;
template <> struct CxT<double> { using T = double2; };
template <> struct CxT<float> { using T = float2; };

// ------------------------------------------------------------------------------------------ index maps
__device__ __forceinline__ int64_t sm_offset(const SliceMap& sm, uint32_t idx) {
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

__device__ __forceinline__ int64_t sm_offset_loc(const SliceMap& sm, uint32_t idx, uint32_t* loc) {
  int64_t off = sm.base;
  uint32_t rem = idx, l = 0;
#pragma unroll
  for (int g = 0; g < kMaxGroups; ++g) {
    if (g < int(sm.ng)) {
      const uint32_t q = (g + 1 < int(sm.ng)) ? magic_div(rem, sm.gmag[g]) : 0u;
      const uint32_t r = rem - q * sm.gdim[g];
      off += int64_t(r) * sm.gstride[g];
      l += r * sm.lmul[g];
      rem = q;
    }
  }
  *loc = l;
  return off;
}

__device__ __forceinline__ int64_t sm64_offset(const SliceMap64& sm, uint64_t idx) {
  int64_t off = sm.base;
  uint64_t rem = idx;
  for (uint32_t g = 0; g < sm.ng; ++g) {
    const uint64_t q = rem / sm.gdim[g];
    off += int64_t(rem - q * sm.gdim[g]) * sm.gstride[g];
    rem = q;
  }
  return off;
}

// ------------------------------------------------------------------------------------------ gate ops
template <typename R, int DT> struct DenseOp { R u[2 * DT * DT]; };
template <typename R, int DT> struct MonoOp { R ph[2 * DT]; int32_t dst[DT]; };

// doff[c] = toff[dst[c]] for monomial gates (filled by the host so no kernel indexes its
// arguments with a run-time value); unused by dense gates.

// put: a result into the state in HBM (ST: streaming store) or into LDS
template <bool ST, typename C>
__device__ __forceinline__ void put(C* p, int64_t i, C v) {
  if constexpr (ST) st_stream(p + i, v);
  else p[i] = v;
}

template <bool ST, typename C, typename R, int DT>
__device__ __forceinline__ void mix_store(C* p, int64_t base, const int64_t* toff, const int64_t*,
                                          const DenseOp<R, DT>& op, const C (&x)[DT]) {
#pragma unroll
  for (int r = 0; r < DT; ++r) {
    R re = R(0), im = R(0);
#pragma unroll
    for (int c = 0; c < DT; ++c) {
      const R ur = op.u[2 * (r * DT + c)], ui = op.u[2 * (r * DT + c) + 1];
      re = fma(ur, x[c].x, re);
      re = fma(-ui, x[c].y, re);
      im = fma(ur, x[c].y, im);
      im = fma(ui, x[c].x, im);
    }
    C y;
    y.x = re;
    y.y = im;
    put<ST>(p, base + toff[r], y);
  }
}

template <bool ST, typename C, typename R, int DT>
__device__ __forceinline__ void mix_store(C* p, int64_t base, const int64_t*, const int64_t* doff,
                                          const MonoOp<R, DT>& op, const C (&x)[DT]) {
#pragma unroll
  for (int c = 0; c < DT; ++c) {
    const R pr = op.ph[2 * c], pi = op.ph[2 * c + 1];
    C y;
    y.x = fma(pr, x[c].x, -pi * x[c].y);
    y.y = fma(pr, x[c].y, pi * x[c].x);
    put<ST>(p, base + doff[c], y);
  }
}

// ------------------------------------------------------------------------------------------ direct
// Controls whose stride is below one 128-byte line leave lines partly active, and controls of
// larger stride that is not a whole number of lines leave the lines at both ends of every active
// run partly active. HBM is written in whole lines here (a partial line costs a read-modify-write),
// so both cases are applied with whole-line writes: amplitudes of inactive slices that share a line
// with active ones are read and written back unchanged, and lines with no active amplitude at all
// are not touched.
enum { kDirectPlain = 0, kDirectPred = 1, kDirectEdge = 2 };

template <typename R, int DT, typename OP>
struct DirectArgs {
  R* psi;
  SliceMap sm;
  int64_t toff[DT];
  int64_t doff[DT];
  OP op;
  // kDirectPred: the low-stride controls are free digits of sm (singleton groups whose lmul weights
  // give their local index); a slice is mixed when that index equals vloc, else written unchanged.
  // Lines holding no amplitude where those controls all have their values are left untouched when
  // lper > 1: line L holds one iff bit (L mod lper) of lmask is set (the pattern of the low control
  // digits repeats every lper lines).
  uint32_t vloc;
  uint32_t lper;
  Magic32 lpm;
  uint64_t lmask;
  // kDirectEdge (every target above the lowest control): sm enumerates the active slices, grouped
  // into blocks of nA = blen consecutive indices (the blen contiguous amplitudes where the lowest
  // control holds its value, all higher digits fixed, each a slice base). Each block gets W lanes,
  // LINE times the most lines a block can touch, taking the amplitudes of those lines in order;
  // lanes outside the block rewrite their amplitudes unchanged (in every target plane whose line
  // holds amplitudes of the block).
  uint32_t nA;
  uint32_t W;
  Magic32 wm;
  uint32_t blen;
  uint32_t nvirt;
  int64_t D;
};

template <typename R> struct LineAmps;   // amplitudes per 128-byte line
template <> struct LineAmps<double> { static constexpr int value = 8; };
template <> struct LineAmps<float> { static constexpr int value = 16; };
template <typename R> constexpr int kLineShift = sizeof(R) == 8 ? 3 : 4;

// Outputs of one slice where every lane stores position y at the same instruction: the mixed
// values where the slice is active, its inputs otherwise (a monomial U picks, for each output row,
// the column whose entry lands there: dst is uniform, so the tests are scalar).
template <typename C, typename R, int DT>
__device__ __forceinline__ void mix_select(const DenseOp<R, DT>& op, const C (&x)[DT], bool act, C (&out)[DT]) {
#pragma unroll
  for (int r = 0; r < DT; ++r) {
    R re = R(0), im = R(0);
#pragma unroll
    for (int c = 0; c < DT; ++c) {
      const R ur = op.u[2 * (r * DT + c)], ui = op.u[2 * (r * DT + c) + 1];
      re = fma(ur, x[c].x, re);
      re = fma(-ui, x[c].y, re);
      im = fma(ur, x[c].y, im);
      im = fma(ui, x[c].x, im);
    }
    out[r].x = act ? re : x[r].x;
    out[r].y = act ? im : x[r].y;
  }
}

template <typename C, typename R, int DT>
__device__ __forceinline__ void mix_select(const MonoOp<R, DT>& op, const C (&x)[DT], bool act, C (&out)[DT]) {
#pragma unroll
  for (int y = 0; y < DT; ++y) out[y] = x[y];
#pragma unroll
  for (int c = 0; c < DT; ++c) {
    const R pr = op.ph[2 * c], pi = op.ph[2 * c + 1];
    C v;
    v.x = fma(pr, x[c].x, -pi * x[c].y);
    v.y = fma(pr, x[c].y, pi * x[c].x);
#pragma unroll
    for (int y = 0; y < DT; ++y)
      if (op.dst[c] == y) {
        out[y].x = act ? v.x : out[y].x;
        out[y].y = act ? v.y : out[y].y;
      }
  }
}

template <typename R, int DT, typename OP, int SPT, int MODE>
__global__ __launch_bounds__(256) void k_slices_direct(DirectArgs<R, DT, OP> a) {
  using C = typename CxT<R>::T;
  C* __restrict__ psi = reinterpret_cast<C*>(a.psi);
  const uint64_t bs = blockDim.x;
  if constexpr (MODE != kDirectPlain) {
    // one slice or edge position per thread; position y of every lane is loaded and stored by
    // one instruction, so each instruction writes whole lines wherever its lanes are consecutive
    int64_t pos;
    bool act = true;
    uint32_t valid = (1u << DT) - 1u;
    if constexpr (MODE == kDirectPred) {
      const uint64_t i = uint64_t(blockIdx.x) * bs + threadIdx.x;
      if (i >= a.sm.count) return;
      uint32_t loc;
      pos = sm_offset_loc(a.sm, uint32_t(i), &loc);
      act = loc == a.vloc;
      if (!act && a.lper > 1) {
        valid = 0;
#pragma unroll
        for (int y = 0; y < DT; ++y) {
          const uint32_t L = uint32_t((pos + a.toff[y]) >> kLineShift<R>);
          if ((a.lmask >> (L - magic_div(L, a.lpm) * a.lper)) & 1u) valid |= 1u << y;
        }
        if (!valid) return;
      }
    } else {
      // the block's lanes walk its lines in order: lane j takes amplitude L0 + j, L0 the start of
      // the line holding the block's first amplitude, so every instruction writes whole lines
      constexpr int LINE = LineAmps<R>::value;
      const uint32_t vi = uint32_t(blockIdx.x) * uint32_t(bs) + threadIdx.x;
      if (vi >= a.nvirt) return;
      const uint32_t b = magic_div(vi, a.wm);
      const int64_t start = sm_offset(a.sm, b * a.nA);
      const int64_t end = start + a.blen - 1;
      pos = (start & ~int64_t(LINE - 1)) + int64_t(vi - b * a.W);
      if (pos > (end | int64_t(LINE - 1))) return;
      act = pos >= start && pos <= end;
      if (!act) {
        // outside the block: rewritten unchanged where its line (in each target plane) holds
        // amplitudes of the block
        valid = 0;
#pragma unroll
        for (int y = 0; y < DT; ++y) {
          const int64_t q = pos + a.toff[y];
          if ((q >> kLineShift<R>) >= ((start + a.toff[y]) >> kLineShift<R>) &&
              (q >> kLineShift<R>) <= ((end + a.toff[y]) >> kLineShift<R>) && q < a.D)
            valid |= 1u << y;
        }
        if (!valid) return;
      }
    }
    C x[DT], out[DT];
#pragma unroll
    for (int y = 0; y < DT; ++y) {
      x[y].x = R(0);
      x[y].y = R(0);
      if (valid & (1u << y)) x[y] = ld_stream(psi + pos + a.toff[y]);
    }
    mix_select<C, R, DT>(a.op, x, act, out);
#pragma unroll
    for (int y = 0; y < DT; ++y)
      if (valid & (1u << y)) st_stream(psi + pos + a.toff[y], out[y]);
  } else {
    const uint64_t first = uint64_t(blockIdx.x) * bs * SPT + threadIdx.x;
    int64_t base[SPT];
    C x[SPT][DT];
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
      const uint64_t i = first + s * bs;
      base[s] = i < a.sm.count ? sm_offset(a.sm, uint32_t(i)) : -1;
    }
#pragma unroll
    for (int s = 0; s < SPT; ++s)
      if (base[s] >= 0) {
#pragma unroll
        for (int y = 0; y < DT; ++y) x[s][y] = ld_stream(psi + base[s] + a.toff[y]);
      }
#pragma unroll
    for (int s = 0; s < SPT; ++s)
      if (base[s] >= 0) mix_store<true, C, R, DT>(psi, base[s], a.toff, a.doff, a.op, x[s]);
  }
}

// Dense gates of d_T = 12 or 16 whose targets all have strides >= run_min: one slice per thread as
// in k_slices_direct, with U (too large for the kernel arguments in complex128) staged in LDS and
// read by broadcast; the slice map and target offsets are staged too, before the first store.
struct LuHead {
  SliceMap sm;
  int64_t toff[16];
  // followed by 2 DT^2 values of R (U, row-major interleaved)
};

template <typename R, int DT>
__global__ __launch_bounds__(256) void k_slices_direct_lu(R* psi_raw, const unsigned char* desc) {
  using C = typename CxT<R>::T;
  __shared__ R su[2 * DT * DT];
  __shared__ SliceMap smap;
  __shared__ int64_t st[DT];
  static_assert(sizeof(SliceMap) % 4 == 0, "slice map copied in 4-byte words");
  const LuHead& h = *reinterpret_cast<const LuHead*>(desc);
  const R* ug = reinterpret_cast<const R*>(desc + sizeof(LuHead));
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < 2u * DT * DT; i += blockDim.x) su[i] = ug[i];
  for (uint32_t i = tid; i < sizeof(SliceMap) / 4; i += blockDim.x)
    reinterpret_cast<uint32_t*>(&smap)[i] = reinterpret_cast<const uint32_t*>(&h.sm)[i];
  if (tid < uint32_t(DT)) st[tid] = h.toff[tid];
  __syncthreads();
  C* __restrict__ psi = reinterpret_cast<C*>(psi_raw);
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + tid;
  if (i >= smap.count) return;
  const int64_t b = sm_offset(smap, uint32_t(i));
  C x[DT];
#pragma unroll
  for (int y = 0; y < DT; ++y) x[y] = ld_stream(psi + b + st[y]);
#pragma unroll
  for (int r = 0; r < DT; ++r) {
    __asm__ volatile("" ::: "memory");   // U is read from LDS here (held in registers it would take hundreds)
    R re = R(0), im = R(0);
#pragma unroll
    for (int c = 0; c < DT; ++c) {
      const R ur = su[2 * (r * DT + c)], ui = su[2 * (r * DT + c) + 1];
      re = fma(ur, x[c].x, re);
      re = fma(-ui, x[c].y, re);
      im = fma(ur, x[c].y, im);
      im = fma(ui, x[c].x, im);
    }
    C yv;
    yv.x = re;
    yv.y = im;
    st_stream(psi + b + st[r], yv);
  }
}

// ------------------------------------------------------------------------------------------ tiled
template <typename R, int DT, typename OP>
struct TileArgs {
  R* psi;
  SliceMap tiles;                 // tile index -> global offset of the tile's origin
  SliceMap inner;                 // slice index inside a tile -> LDS index of its y = 0 amplitude
  uint32_t BL;                    // run length (amplitudes of the low suffix)
  uint32_t dH;                    // number of runs (product of the high targets' dims)
  Magic32 blm;                    // division by BL
  int64_t hoff[kMaxTileRuns];     // global offset of run h from the tile origin
  int64_t toff[DT];               // LDS offset of target combination y
  int64_t doff[DT];               // monomial: LDS offset of the row column y moves to
  uint32_t nsc;                   // controls inside the suffix that the tile leaves out, and for
  Magic32 scm[kMaxTileCtl];       // each, by increasing stride s: division by s,
  uint32_t scmul[kMaxTileCtl];    // s (d_c - 1) and
  uint32_t scadd[kMaxTileCtl];    // v s (v: the control value)
  OP op;
};

// Dense gates read U from LDS in the tile kernel. Left to the compiler, its 2 d_T^2 values join the
// slice maps in the scalar registers, which overflow, and the mix then spends more instructions
// reading spilled values back than multiplying. Each workgroup copies U from the kernel argument
// segment (one vector load per thread, no upload) into LDS before its first tile.
constexpr int kTileLdsU = 2;
template <typename OP> struct DenseDim { static constexpr int value = 0; };
template <typename R, int DT> struct DenseDim<DenseOp<R, DT>> { static constexpr int value = DT; };

// Offset inside the run of the staged amplitude w: each left-out control digit is re-inserted at
// its value, smallest stride first (w = q s + r becomes q s d_c + v s + r).
template <typename A>
__device__ __forceinline__ uint32_t tile_expand(const A& a, uint32_t w) {
#pragma unroll
  for (int j = 0; j < kMaxTileCtl; ++j)
    if (j < int(a.nsc)) w += magic_div(w, a.scm[j]) * a.scmul[j] + a.scadd[j];
  return w;
}

// Amplitudes a thread moves per tile: the tile holds at most 256 * kTileEpt<R> amplitudes.
template <typename R> struct TileEpt;
template <> struct TileEpt<double> { static constexpr int value = 8; };
template <> struct TileEpt<float> { static constexpr int value = 16; };

template <typename R, int DT, typename OP>
__global__ __launch_bounds__(256) void k_slices_tiled(TileArgs<R, DT, OP> a) {
  using C = typename CxT<R>::T;
  constexpr int EPT = TileEpt<R>::value;
  constexpr int kUL = DenseDim<OP>::value >= kTileLdsU ? 2 * DT * DT : 0;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int64_t s_hoff[kMaxTileRuns];
  __shared__ R su[kUL > 0 ? kUL : 1];
  C* lds = reinterpret_cast<C*>(lds_raw);
  C* __restrict__ psi = reinterpret_cast<C*>(a.psi);
  const uint32_t bs = blockDim.x, tid = threadIdx.x;
  const uint32_t E = a.BL * a.dH;
#pragma unroll
  for (int h = 0; h < kMaxTileRuns; ++h)
    if (int(tid) == h) s_hoff[h] = a.hoff[h];
  if constexpr (kUL > 0) {
    const R* ug = a.op.u;   // read in place from the kernel argument segment
    for (uint32_t i = tid; i < uint32_t(kUL); i += bs) su[i] = ug[i];
  }
  __syncthreads();
  for (uint32_t tile = blockIdx.x; tile < a.tiles.count; tile += gridDim.x) {
    const int64_t g0 = sm_offset(a.tiles, tile);
    // The per-element run and LDS indices are recomputed in the load and in the store stage from
    // opaque copies of the thread index: kept live across the LDS mix they would take about
    // 3 EPT registers and cut the workgroups per CU for the wider gates.
    uint32_t tl = tid;
    __asm__ volatile("" : "+v"(tl));
    // every load of the tile is issued before the first LDS write
    // (real and imaginary parts in separate scalar arrays so they stay in registers)
    R vr[EPT], vi[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const uint32_t idx = tl + e * bs;
      if (idx < E) {
        const uint32_t h = magic_div(idx, a.blm);
        const C t = ld_stream(psi + (g0 + s_hoff[h] + tile_expand(a, idx - h * a.BL)));
        vr[e] = t.x;
        vi[e] = t.y;
      }
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const uint32_t idx = tl + e * bs;
      if (idx < E) {
        C t;
        t.x = vr[e];
        t.y = vi[e];
        lds[idx] = t;
      }
    }
    __syncthreads();
    for (uint32_t j = tid; j < a.inner.count; j += bs) {
      const int64_t b = sm_offset(a.inner, j);
      C x[DT];
#pragma unroll
      for (int y = 0; y < DT; ++y) x[y] = lds[b + a.toff[y]];
      if constexpr (kUL > 0) {
#pragma unroll
        for (int r = 0; r < DT; ++r) {
          __asm__ volatile("" ::: "memory");   // U is read from LDS row by row, not held in registers
          R re = R(0), im = R(0);
#pragma unroll
          for (int c = 0; c < DT; ++c) {
            const R ur = su[2 * (r * DT + c)], ui = su[2 * (r * DT + c) + 1];
            re = fma(ur, x[c].x, re);
            re = fma(-ui, x[c].y, re);
            im = fma(ur, x[c].y, im);
            im = fma(ui, x[c].x, im);
          }
          C yv;
          yv.x = re;
          yv.y = im;
          lds[b + a.toff[r]] = yv;
        }
      } else {
        mix_store<false, C, R, DT>(lds, b, a.toff, a.doff, a.op, x);
      }
    }
    __syncthreads();
    uint32_t ts = tid;
    __asm__ volatile("" : "+v"(ts));
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const uint32_t idx = ts + e * bs;
      if (idx < E) {
        const C t = lds[idx];
        vr[e] = t.x;
        vi[e] = t.y;
      }
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const uint32_t idx = ts + e * bs;
      if (idx < E) {
        const uint32_t h = magic_div(idx, a.blm);
        C t;
        t.x = vr[e];
        t.y = vi[e];
        st_stream(psi + (g0 + s_hoff[h] + tile_expand(a, idx - h * a.BL)), t);
      }
    }
    if (tile + gridDim.x < a.tiles.count) __syncthreads();
  }
}

// ------------------------------------------------------------------------------------------ diagonal
template <typename R>
struct DiagArgs {
  R* psi;
  SliceMap sm;                     // over all non-control qudits; targets are singleton groups
  R ph[2 * kMaxInlineTable];       // phase of target combination loc
};

template <typename R, int SPT>
__global__ __launch_bounds__(256) void k_diag(DiagArgs<R> a) {
  using C = typename CxT<R>::T;
  C* __restrict__ psi = reinterpret_cast<C*>(a.psi);
  const uint64_t bs = blockDim.x;
  const uint64_t first = uint64_t(blockIdx.x) * bs * SPT + threadIdx.x;
  int64_t off[SPT];
  uint32_t loc[SPT];
  C x[SPT];
#pragma unroll
  for (int s = 0; s < SPT; ++s) {
    const uint64_t i = first + s * bs;
    off[s] = i < a.sm.count ? sm_offset_loc(a.sm, uint32_t(i), &loc[s]) : -1;
  }
#pragma unroll
  for (int s = 0; s < SPT; ++s)
    if (off[s] >= 0) x[s] = ld_stream(psi + off[s]);
#pragma unroll
  for (int s = 0; s < SPT; ++s)
    if (off[s] >= 0) {
      const R pr = a.ph[2 * loc[s]], pi = a.ph[2 * loc[s] + 1];
      C y;
      y.x = fma(pr, x[s].x, -pi * x[s].y);
      y.y = fma(pr, x[s].y, pi * x[s].x);
      st_stream(psi + off[s], y);
    }
}

// ------------------------------------------------------------------------------------------ generic
struct GenericHead {
  SliceMap64 sm;
  int32_t dT;
  int32_t nsw;        // slices per workgroup iteration
  // followed by int64_t toff[dT] and then 2 dT^2 values of R (U, row-major interleaved)
};

template <typename R>
__global__ __launch_bounds__(256) void k_dense_generic(R* psi_raw, const unsigned char* desc) {
  using C = typename CxT<R>::T;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  C* xs = reinterpret_cast<C*>(lds_raw);
  const GenericHead& h = *reinterpret_cast<const GenericHead*>(desc);
  // the slice map is read into LDS before the first store (read later from global memory it would
  // be fetched again by vector loads, the stores could alias it)
  __shared__ SliceMap64 smap;
  static_assert(sizeof(SliceMap64) % 4 == 0, "slice map copied in 4-byte words");
  for (uint32_t i = threadIdx.x; i < sizeof(SliceMap64) / 4; i += blockDim.x)
    reinterpret_cast<uint32_t*>(&smap)[i] = reinterpret_cast<const uint32_t*>(&h.sm)[i];
  const int64_t* toff = reinterpret_cast<const int64_t*>(desc + sizeof(GenericHead));
  const R* U = reinterpret_cast<const R*>(desc + sizeof(GenericHead) + sizeof(int64_t) * h.dT);
  C* psi = reinterpret_cast<C*>(psi_raw);
  const uint32_t dT = uint32_t(h.dT), nsw = uint32_t(h.nsw), tot = dT * nsw;
  const uint64_t count = h.sm.count;
  __syncthreads();
  for (uint64_t s0 = uint64_t(blockIdx.x) * nsw; s0 < count; s0 += uint64_t(gridDim.x) * nsw) {
    for (uint32_t e = threadIdx.x; e < tot; e += blockDim.x) {
      const uint32_t j = e / dT, y = e - j * dT;
      if (s0 + j < count) xs[e] = ld_stream(psi + (sm64_offset(smap, s0 + j) + toff[y]));
    }
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < tot; e += blockDim.x) {
      const uint32_t j = e / dT, row = e - j * dT;
      if (s0 + j >= count) continue;
      R re = R(0), im = R(0);
      const R* u = U + 2 * size_t(row) * dT;
      const C* x = xs + j * dT;
      for (uint32_t c = 0; c < dT; ++c) {
        re = fma(u[2 * c], x[c].x, re);
        re = fma(-u[2 * c + 1], x[c].y, re);
        im = fma(u[2 * c], x[c].y, im);
        im = fma(u[2 * c + 1], x[c].x, im);
      }
      C y;
      y.x = re;
      y.y = im;
      st_stream(psi + (sm64_offset(smap, s0 + j) + toff[row]), y);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------------ gemm
// Dense gates with kGemmMin <= d_T <= kGemmMax on registers below 2^32 amplitudes: per tile of ns
// slices, Y = U X as a small complex GEMM. U (zero-padded to dP = d_T rounded up to a multiple of 4,
// rows kGemmPad elements apart so the rows a wavefront reads fall in different banks) and the
// tile's X (dP rows x ns slices) sit in LDS; each thread accumulates a 4 x 4 block of outputs in
// registers; the results go back through LDS, so loads and stores both run over consecutive
// slices. Workgroups are persistent and stage U once.
constexpr int kGemmMin = 10;
constexpr int kGemmMax = 64;
constexpr int kGemmOut = 4096;        // outputs per tile (dP x ns), 16 per thread
// The tile moves between HBM and LDS element by element in one of two orders: slices fastest (the
// free digits hold the smallest stride), or target combinations fastest in ascending offset (a
// target holds the smallest stride), so that consecutive lanes touch neighbouring amplitudes.
struct GemmHead {
  SliceMap sm;                        // slices: the non-target digits (controls fixed)
  Magic32 nsm;                        // division by ns
  Magic32 dpm;                        // division by dP
  int32_t dT, dP, ns, yfast;
  // followed by int64_t toff[dT], int32_t yord[dP] (target combinations by ascending offset, then
  // the padding rows) and 2 dP^2 values of R (U zero-padded, row-major)
};

template <typename R>
__global__ __launch_bounds__(256) void k_dense_gemm(R* psi_raw, const unsigned char* desc) {
  using C = typename CxT<R>::T;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const GemmHead& h = *reinterpret_cast<const GemmHead*>(desc);
  // the head is read into locals and LDS before the first store: read later from global memory it
  // would be fetched again by vector loads (the stores could alias it)
  __shared__ SliceMap smap;
  static_assert(sizeof(SliceMap) % 4 == 0, "slice map copied in 4-byte words");
  for (uint32_t i = threadIdx.x; i < sizeof(SliceMap) / 4; i += blockDim.x)
    reinterpret_cast<uint32_t*>(&smap)[i] = reinterpret_cast<const uint32_t*>(&h.sm)[i];
  const Magic32 nsm = h.nsm, dpm = h.dpm;
  const uint32_t dT = uint32_t(h.dT), dP = uint32_t(h.dP), ns = uint32_t(h.ns), ldu = dP + 1;
  const uint32_t count = h.sm.count;
  C* __restrict__ psi = reinterpret_cast<C*>(psi_raw);
  C* xs = reinterpret_cast<C*>(lds_raw);                        // dP x ns, element (y, j) at y ns + j
  C* us = xs + dP * ns;                                         // dP x dP, row stride ldu
  int64_t* sb = reinterpret_cast<int64_t*>(us + dP * ldu);     // ns slice bases
  int64_t* to = sb + ns;                                        // dT target offsets
  int32_t* yo = reinterpret_cast<int32_t*>(to + dT);            // dP rows in memory order
  const int64_t* tg = reinterpret_cast<const int64_t*>(desc + sizeof(GemmHead));
  const int32_t* yg = reinterpret_cast<const int32_t*>(desc + sizeof(GemmHead) + sizeof(int64_t) * dT);
  const R* ug = reinterpret_cast<const R*>(desc + sizeof(GemmHead) + sizeof(int64_t) * dT + sizeof(int32_t) * dP);
  const bool yfast = h.yfast != 0;
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < dP * dP; i += blockDim.x) {
    const uint32_t r = i / dP, c = i - r * dP;
    C v;
    v.x = ug[2 * i];
    v.y = ug[2 * i + 1];
    us[r * ldu + c] = v;
  }
  for (uint32_t i = tid; i < dT; i += blockDim.x) to[i] = tg[i];
  for (uint32_t i = tid; i < dP; i += blockDim.x) yo[i] = yg[i];
  const uint32_t rbn = dP / 4, nblk = rbn * (ns / 4);
  const uint32_t rb = tid % rbn, kb = tid / rbn;                // this thread's 4 x 4 output block
  const uint32_t ntiles = (count + ns - 1) / ns;
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint32_t s0 = tile * ns;
    __syncthreads();   // U staged; the previous tile is stored
    for (uint32_t j = tid; j < ns; j += blockDim.x) sb[j] = s0 + j < count ? sm_offset(smap, s0 + j) : int64_t(-1);
    __syncthreads();
    // every load of the tile in flight before the first LDS write (at most kGemmOut / 256 each)
    {
      constexpr int EPT = kGemmOut / 256;
      const uint32_t tot = dP * ns;
      C v[EPT];
      uint32_t at[EPT];
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const uint32_t e = tid + uint32_t(k) * 256u;
        v[k].x = R(0);
        v[k].y = R(0);
        at[k] = 0xFFFFFFFFu;
        if (e < tot) {
          uint32_t y, j;
          if (yfast) {
            j = magic_div(e, dpm);
            y = uint32_t(yo[e - j * dP]);
          } else {
            y = magic_div(e, nsm);
            j = e - y * ns;
          }
          at[k] = y * ns + j;
          if (y < dT && sb[j] >= 0) v[k] = ld_stream(psi + (sb[j] + to[y]));
        }
      }
#pragma unroll
      for (int k = 0; k < EPT; ++k)
        if (at[k] != 0xFFFFFFFFu) xs[at[k]] = v[k];
    }
    __syncthreads();
    C acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        acc[i][k].x = R(0);
        acc[i][k].y = R(0);
      }
    if (tid < nblk) {
      const C* ur = us + 4 * rb * ldu;
      const C* xc = xs + 4 * kb;
      for (uint32_t c = 0; c < dP; ++c) {
        C u[4], x[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) u[i] = ur[i * ldu + c];
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = xc[c * ns + k];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            acc[i][k].x = fma(u[i].x, x[k].x, acc[i][k].x);
            acc[i][k].x = fma(-u[i].y, x[k].y, acc[i][k].x);
            acc[i][k].y = fma(u[i].x, x[k].y, acc[i][k].y);
            acc[i][k].y = fma(u[i].y, x[k].x, acc[i][k].y);
          }
      }
    }
    __syncthreads();   // every product has read X
    if (tid < nblk) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) xs[(4 * rb + i) * ns + 4 * kb + k] = acc[i][k];
    }
    __syncthreads();
    for (uint32_t e = tid; e < dP * ns; e += blockDim.x) {
      uint32_t y, j;
      if (yfast) {
        j = magic_div(e, dpm);
        y = uint32_t(yo[e - j * dP]);
      } else {
        y = magic_div(e, nsm);
        j = e - y * ns;
      }
      if (y < dT && sb[j] >= 0) st_stream(psi + (sb[j] + to[y]), xs[y * ns + j]);
    }
  }
}

// ------------------------------------------------------------------------------------------ launch helpers
// Name of the kernel instance the calling thread's last gate launch used (qd_last_kernel).
static thread_local const char* g_last_kernel = "";

template <typename R> constexpr const char* real_name() { return sizeof(R) == 8 ? "double" : "float"; }
template <typename OP> struct OpName;
template <typename R, int DT> struct OpName<DenseOp<R, DT>> { static constexpr const char* value = "DenseOp"; };
template <typename R, int DT> struct OpName<MonoOp<R, DT>> { static constexpr const char* value = "MonoOp"; };

// "<kernel><R, DT[, Op<R, DT>][, SPT, mode]>", formatted once per instance
enum { kKnDirect, kKnTiled, kKnDiag, kKnGeneric, kKnGemm, kKnLu };
template <int KIND, typename R, int DT = 0, typename OP = void, int SPT = 0, int MODE = 0>
static const char* label() {
  static thread_local char buf[160] = {0};
  if (!buf[0]) {
    static const char* kn[] = {"k_slices_direct", "k_slices_tiled", "k_diag", "k_dense_generic", "k_dense_gemm",
                               "k_slices_direct_lu"};
    static const char* modes[] = {"plain", "pred", "edge"};
    const char* rn = real_name<R>();
    if constexpr (KIND == kKnDirect)
      std::snprintf(buf, sizeof(buf), "%s<%s, %d, %s<%s, %d>, %d, %s>", kn[KIND], rn, DT, OpName<OP>::value, rn, DT, SPT,
                    modes[MODE]);
    else if constexpr (KIND == kKnTiled)
      std::snprintf(buf, sizeof(buf), "%s<%s, %d, %s<%s, %d>>", kn[KIND], rn, DT, OpName<OP>::value, rn, DT);
    else if constexpr (KIND == kKnLu)
      std::snprintf(buf, sizeof(buf), "%s<%s, %d>", kn[KIND], rn, DT);
    else
      std::snprintf(buf, sizeof(buf), "%s<%s>", kn[KIND], rn);
  }
  return buf;
}

static inline unsigned grid_for(uint64_t items, uint64_t per_block) {
  const uint64_t g = (items + per_block - 1) / per_block;
  return unsigned(std::max<uint64_t>(1, g));
}

static int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, what);
  return QD_OK;
}

// Which lines of `line` amplitudes hold an amplitude where every control of stride below one line
// has its value. Those control digits repeat with period P = lcm(s_c d_c), so the lines repeat with
// period lcm(P, line) / line; for a period of 2..64 lines, *per is set to it and bit j of *mask
// tells whether line j of a period holds such an amplitude (else *per = 1: treat every line so).
static void line_pattern(const Register& r, const GatePlan& p, int64_t line, uint32_t* per, uint64_t* mask) {
  *per = 1;
  *mask = 1;
  uint64_t P = 1;
  for (int j = 0; j < p.m; ++j) {
    const int c = p.controls[j];
    if (r.strides[c] < line) P = std::lcm(P, uint64_t(r.strides[c]) * uint64_t(r.dims[c]));
  }
  const uint64_t per_lines = std::lcm(P, uint64_t(line)) / uint64_t(line);
  if (per_lines < 2 || per_lines > 64) return;
  uint64_t m = 0;
  for (uint64_t L = 0; L < per_lines; ++L)
    for (uint64_t i = L * uint64_t(line); i < (L + 1) * uint64_t(line); ++i) {
      bool all = true;
      for (int j = 0; j < p.m && all; ++j) {
        const int c = p.controls[j];
        if (r.strides[c] < line) all = (i / uint64_t(r.strides[c])) % uint64_t(r.dims[c]) == uint64_t(p.cvals[j]);
      }
      if (all) {
        m |= uint64_t(1) << L;
        break;
      }
    }
  if (m == (per_lines == 64 ? ~uint64_t(0) : (uint64_t(1) << per_lines) - 1)) return;   // every line
  *per = uint32_t(per_lines);
  *mask = m;
}

// target offsets: y in mixed radix over the targets in listed order, t_0 most significant
static void target_offsets(const Register& r, const GatePlan& p, int64_t* toff) {
  for (int y = 0; y < p.dT; ++y) {
    int rem = y;
    int64_t off = 0;
    for (int j = p.k - 1; j >= 0; --j) {
      const int d = r.dims[p.targets[j]];
      off += int64_t(rem % d) * r.strides[p.targets[j]];
      rem /= d;
    }
    toff[y] = off;
  }
}

template <typename R, int DT>
static void fill_dense(const GatePlan& p, DenseOp<R, DT>* op) {
  for (int i = 0; i < 2 * DT * DT; ++i) op->u[i] = R(p.U[i]);
}
template <typename R, int DT>
static void fill_mono(const GatePlan& p, MonoOp<R, DT>* op) {
  for (int i = 0; i < DT; ++i) {
    op->dst[i] = p.dst[i];
    op->ph[2 * i] = R(p.ph[2 * i]);
    op->ph[2 * i + 1] = R(p.ph[2 * i + 1]);
  }
}

// LDS tile geometry: the low suffix L = {pq, ..., n-1} of the register holds every target whose
// stride is below run_min and is grown towards longer contiguous runs while the tile (dH runs of
// BL amplitudes) fits the LDS budget. Controls inside L (at most kMaxTileCtl; their strides are at
// least one 128-byte line, smaller ones having been folded into the targets) are left out of the
// tile: it stages only the amplitudes whose control digits match, so a control that falls inside
// L costs 1/d_c of a pass as it does above L. Returns false when no target is low (the direct
// kernel applies) or the tile would not fit.
bool tile_geometry(const Register& r, const GatePlan& p, int prec, TileGeom* g) {
  const TuneParams& tp = tune();
  int64_t min_stride = INT64_MAX;
  int min_t = -1;
  for (int j = 0; j < p.k; ++j)
    if (r.strides[p.targets[j]] < min_stride) {
      min_stride = r.strides[p.targets[j]];
      min_t = p.targets[j];
    }
  const TuneEntry e = entry_for(prec, min_stride);
  if (!e.tiled) return false;
  {
    // Controls inside a line that leave whole lines without a matching amplitude: the predicated
    // direct kernel skips those lines and the tile kernel would move them. With every target at
    // least a line apart the direct kernel's lanes still take whole lines, so it runs such gates.
    const int64_t line = prec == QD_C128 ? 8 : 16;
    uint32_t per = 1;
    uint64_t mask = 1;
    if (min_stride >= line) line_pattern(r, p, line, &per, &mask);
    if (per > 1) return false;
  }
  int low_idx = min_t;
  for (int j = 0; j < p.k; ++j)
    if (r.strides[p.targets[j]] < tp.run_min) low_idx = std::min(low_idx, int(p.targets[j]));
  const uint64_t ept = prec == QD_C128 ? TileEpt<double>::value : TileEpt<float>::value;
  const uint64_t emax = std::min<uint64_t>(uint64_t(e.tile_elems) * (prec == QD_C128 ? 1u : 2u),
                                           uint64_t(e.block) * ept);
  const int64_t line = prec == QD_C128 ? 8 : 16;   // amplitudes per 128-byte line
  bool is_t[QD_MAX_QUDITS] = {}, is_c[QD_MAX_QUDITS] = {};
  for (int j = 0; j < p.k; ++j) is_t[p.targets[j]] = true;
  for (int j = 0; j < p.m; ++j) is_c[p.controls[j]] = r.strides[p.controls[j]] >= line;
  auto grow = [&](bool compact) -> bool {
    int pq = low_idx, nsc = 0;
    uint64_t BL = 1, dH = 1;
    for (int i = pq; i < r.n; ++i) {
      if (compact && is_c[i]) ++nsc;
      else BL *= uint64_t(r.dims[i]);
    }
    if (nsc > kMaxTileCtl) return false;
    for (int i = 0; i < pq; ++i)
      if (is_t[i]) dH *= r.dims[i];
    while (pq > 0) {
      const int q = pq - 1;
      const bool drop = compact && is_c[q];
      if (drop && nsc == kMaxTileCtl) break;
      const uint64_t nBL = drop ? BL : BL * r.dims[q];
      const uint64_t ndH = is_t[q] ? dH / r.dims[q] : dH;
      if (nBL * ndH > emax) break;
      pq = q;
      BL = nBL;
      dH = ndH;
      nsc += drop ? 1 : 0;
    }
    if (dH > uint64_t(kMaxTileRuns) || BL * dH > emax) return false;
    g->pq = pq;
    g->BL = BL;
    g->dH = dH;
    g->nsc = 0;
    for (int i = r.n - 1; i >= pq && compact; --i)
      if (is_c[i]) g->sc[g->nsc++] = i;
    return true;
  };
  return grow(true) || grow(false);
}

int route_gate(const Register& r, int prec, const GatePlan& p) {
  const bool fast = uint64_t(r.D) <= 0xFFFFFFFFull;
  if (!fast) return QD_ROUTE_GENERIC;
  if (p.cls == QD_CLASS_DIAGONAL && p.dT <= kMaxInlineTable) return QD_ROUTE_DIAG;
  const bool mono = p.cls == QD_CLASS_MONOMIAL &&
                    (p.dT <= 9 || p.dT == 12 || p.dT == 16);
  const bool dense = p.cls != QD_CLASS_DIAGONAL && p.dT <= kMaxInlineDense;
  if (!mono && !dense) {
    if (p.dT < kGemmMin || p.dT > kGemmMax) return QD_ROUTE_GENERIC;
    // d_T = 12 or 16 with every target stride at or above the tiling threshold: one slice per thread
    if (p.dT == 12 || p.dT == 16) {
      int64_t tmin = INT64_MAX;
      for (int j = 0; j < p.k; ++j) tmin = std::min<int64_t>(tmin, r.strides[p.targets[j]]);
      if (tmin >= tune().run_min) return QD_ROUTE_DIRECT;
    }
    return QD_ROUTE_GEMM;
  }
  TileGeom g;
  return tile_geometry(r, p, prec, &g) ? QD_ROUTE_TILED : QD_ROUTE_DIRECT;
}

template <int DT>
static void fill_doff(const GatePlan& p, const int64_t* toff, int64_t* doff) {
  for (int c = 0; c < DT; ++c) doff[c] = p.dst.empty() ? 0 : toff[p.dst[c]];
}

template <typename R, int DT, typename OP>
static int launch_slices(qd_state* s, const GatePlan& p, const OP& op) {
  const Register& r = s->reg;
  const TuneParams& tp = tune();
  int role[QD_MAX_QUDITS] = {};
  for (int j = 0; j < p.k; ++j) role[p.targets[j]] = 1;
  for (int j = 0; j < p.m; ++j) role[p.controls[j]] = 1;

  int64_t min_stride = INT64_MAX;
  for (int j = 0; j < p.k; ++j) min_stride = std::min<int64_t>(min_stride, r.strides[p.targets[j]]);
  const TuneEntry ent = entry_for(s->prec, min_stride);
  TileGeom tg;
  if (tile_geometry(r, p, s->prec, &tg)) {
    const int pq = tg.pq;
    const uint64_t BL = tg.BL, dH = tg.dH;
    {
      TileArgs<R, DT, OP> a;
      std::memset(&a, 0, sizeof(a));
      a.psi = reinterpret_cast<R*>(s->data);
      a.op = op;
      a.BL = uint32_t(BL);
      a.dH = uint32_t(dH);
      a.blm = make_magic32(uint32_t(BL));
      // LDS strides of the suffix: the register's, with the left-out controls' digits removed
      bool out[QD_MAX_QUDITS] = {};
      for (int j = 0; j < tg.nsc; ++j) out[tg.sc[j]] = true;
      Register lr = r;
      {
        int64_t st = 1;
        for (int i = r.n - 1; i >= pq; --i) {
          lr.strides[i] = st;
          if (!out[i]) st *= r.dims[i];
        }
      }
      int64_t tbase = 0, ibase = 0;
      for (int j = 0; j < p.m; ++j) {
        const int c = p.controls[j];
        if (c < pq) tbase += int64_t(p.cvals[j]) * r.strides[c];
        else if (!out[c]) ibase += int64_t(p.cvals[j]) * lr.strides[c];
      }
      a.nsc = uint32_t(tg.nsc);
      for (int j = 0; j < tg.nsc; ++j) {
        const int c = tg.sc[j];
        int v = 0;
        for (int q = 0; q < p.m; ++q)
          if (p.controls[q] == c) v = p.cvals[q];
        a.scm[j] = make_magic32(uint32_t(r.strides[c]));
        a.scmul[j] = uint32_t(r.strides[c] * (r.dims[c] - 1));
        a.scadd[j] = uint32_t(int64_t(v) * r.strides[c]);
      }
      int rc = fill_slicemap(make_groups(r, role, nullptr, 0, pq), tbase, &a.tiles);
      if (rc) return rc;
      rc = fill_slicemap(make_groups(lr, role, nullptr, pq, r.n), ibase, &a.inner);
      if (rc) return rc;
      // run offsets: h in mixed radix over the high targets in listed order
      int hmul[QD_MAX_QUDITS] = {};
      {
        int m = 1;
        for (int j = p.k - 1; j >= 0; --j)
          if (p.targets[j] < pq) {
            hmul[j] = m;
            m *= r.dims[p.targets[j]];
          }
      }
      for (uint32_t h = 0; h < a.dH; ++h) {
        int64_t off = 0;
        for (int j = 0; j < p.k; ++j)
          if (p.targets[j] < pq) off += int64_t((h / hmul[j]) % r.dims[p.targets[j]]) * r.strides[p.targets[j]];
        a.hoff[h] = off;
      }
      for (int y = 0; y < DT; ++y) {
        int rem = y;
        int64_t off = 0;
        for (int j = p.k - 1; j >= 0; --j) {
          const int t = p.targets[j];
          const int dg = rem % r.dims[t];
          rem /= r.dims[t];
          off += t < pq ? int64_t(dg) * hmul[j] * int64_t(BL) : int64_t(dg) * lr.strides[t];
        }
        a.toff[y] = off;
      }
      fill_doff<DT>(p, a.toff, a.doff);
      if (a.tiles.count == 0 || a.inner.count == 0) return QD_OK;
      const size_t lds = size_t(BL * dH) * sizeof(R) * 2;
      // workgroups walk the tiles; at most 2^22 of them keep the grid inside 32-bit work-item counts
      const unsigned grid = unsigned(std::min<uint64_t>(a.tiles.count, uint64_t(1) << 22));
      hipLaunchKernelGGL((k_slices_tiled<R, DT, OP>), dim3(grid), dim3(ent.block), lds, s->stream, a);
      g_last_kernel = label<kKnTiled, R, DT, OP>();
      return check_launch("k_slices_tiled");
    }
  }

  // ---- direct: one slice per thread
  DirectArgs<R, DT, OP> a;
  std::memset(&a, 0, sizeof(a));
  a.psi = reinterpret_cast<R*>(s->data);
  a.op = op;
  const int64_t line = LineAmps<R>::value;
  // controls below one line are free digits of the slice map, tested per slice (kDirectPred)
  uint32_t lmul[QD_MAX_QUDITS] = {};
  int nlow = 0, c0 = -1;
  {
    uint32_t w = 1;
    for (int j = p.m - 1; j >= 0; --j) {
      const int c = p.controls[j];
      if (r.strides[c] < line) {
        role[c] = 2;
        lmul[c] = w;
        a.vloc += uint32_t(p.cvals[j]) * w;
        w *= uint32_t(r.dims[c]);
        ++nlow;
      } else if (c0 < 0 || r.strides[c] < r.strides[c0]) {
        c0 = c;
      }
    }
  }
  int64_t base = 0;
  for (int j = 0; j < p.m; ++j)
    if (role[p.controls[j]] == 1) base += int64_t(p.cvals[j]) * r.strides[p.controls[j]];
  int rc = fill_slicemap(make_groups(r, role, nlow ? lmul : nullptr, 0, r.n), base, &a.sm);
  if (rc) return rc;
  target_offsets(r, p, a.toff);
  fill_doff<DT>(p, a.toff, a.doff);
  if (a.sm.count == 0) return QD_OK;
  const int bs = ent.block;
  if (nlow) {
    line_pattern(r, p, line, &a.lper, &a.lmask);
    if (a.lper > 1) a.lpm = make_magic32(a.lper);
    hipLaunchKernelGGL((k_slices_direct<R, DT, OP, 1, kDirectPred>), dim3(grid_for(a.sm.count, uint64_t(bs))), dim3(bs), 0,
                       s->stream, a);
    g_last_kernel = label<kKnDirect, R, DT, OP, 1, kDirectPred>();
    return check_launch("k_slices_direct");
  }
  // the lowest control's active runs end inside lines: edge lanes rewrite the rest of those lines
  bool above = c0 >= 0;
  for (int j = 0; j < p.k && above; ++j) above = r.strides[p.targets[j]] > r.strides[c0];
  if (above && r.strides[c0] % line != 0) {
    const int64_t sc = r.strides[c0];
    uint64_t nA = 1;   // every qudit below the control is free (the targets are above it)
    for (int i = r.n - 1; i >= 0 && r.strides[i] < sc; --i) nA *= uint64_t(r.dims[i]);
    const uint64_t nblk = a.sm.count / nA;
    const uint64_t W = (uint64_t(sc) + 2 * uint64_t(line) - 2) / uint64_t(line) * uint64_t(line);   // lines a block can touch
    if (nblk * nA == a.sm.count && nblk * W <= 0xFFFFFFFFull) {
      a.nA = uint32_t(nA);
      a.W = uint32_t(W);
      a.wm = make_magic32(uint32_t(W));
      a.blen = uint32_t(sc);
      a.nvirt = uint32_t(nblk * W);
      a.D = r.D;
      hipLaunchKernelGGL((k_slices_direct<R, DT, OP, 1, kDirectEdge>), dim3(grid_for(a.nvirt, uint64_t(bs))), dim3(bs), 0,
                         s->stream, a);
      g_last_kernel = label<kKnDirect, R, DT, OP, 1, kDirectEdge>();
      return check_launch("k_slices_direct");
    }
  }
  // Several slices per thread only up to d_T = 4: beyond, two slices' operands and the gate's
  // kernel arguments overflow the scalar registers and the spilled values are read back per FMA.
  if (ent.spt >= 4 && DT <= 4) {
    hipLaunchKernelGGL((k_slices_direct<R, DT, OP, 4, kDirectPlain>), dim3(grid_for(a.sm.count, uint64_t(bs) * 4)), dim3(bs),
                       0, s->stream, a);
    g_last_kernel = label<kKnDirect, R, DT, OP, 4, kDirectPlain>();
  } else if (ent.spt >= 2 && DT <= 4) {
    hipLaunchKernelGGL((k_slices_direct<R, DT, OP, 2, kDirectPlain>), dim3(grid_for(a.sm.count, uint64_t(bs) * 2)), dim3(bs),
                       0, s->stream, a);
    g_last_kernel = label<kKnDirect, R, DT, OP, 2, kDirectPlain>();
  } else {
    hipLaunchKernelGGL((k_slices_direct<R, DT, OP, 1, kDirectPlain>), dim3(grid_for(a.sm.count, uint64_t(bs))), dim3(bs), 0,
                       s->stream, a);
    g_last_kernel = label<kKnDirect, R, DT, OP, 1, kDirectPlain>();
  }
  return check_launch("k_slices_direct");
}

template <typename R, int DT>
static int launch_dense_t(qd_state* s, const GatePlan& p) {
  DenseOp<R, DT> op;
  fill_dense<R, DT>(p, &op);
  return launch_slices<R, DT>(s, p, op);
}

template <typename R, int DT>
static int launch_mono_t(qd_state* s, const GatePlan& p) {
  MonoOp<R, DT> op;
  fill_mono<R, DT>(p, &op);
  return launch_slices<R, DT>(s, p, op);
}

template <typename R>
static int launch_diag(qd_state* s, const GatePlan& p) {
  const Register& r = s->reg;
  int role[QD_MAX_QUDITS] = {};
  uint32_t lmul[QD_MAX_QUDITS] = {};
  uint32_t m = 1;
  for (int j = p.k - 1; j >= 0; --j) {
    role[p.targets[j]] = 2;
    lmul[p.targets[j]] = m;
    m *= uint32_t(r.dims[p.targets[j]]);
  }
  for (int j = 0; j < p.m; ++j) role[p.controls[j]] = 1;
  DiagArgs<R> a;
  std::memset(&a, 0, sizeof(a));
  a.psi = reinterpret_cast<R*>(s->data);
  int64_t base = 0;
  for (int j = 0; j < p.m; ++j) base += int64_t(p.cvals[j]) * r.strides[p.controls[j]];
  int rc = fill_slicemap(make_groups(r, role, lmul, 0, r.n), base, &a.sm);
  if (rc) return rc;
  for (int i = 0; i < 2 * p.dT; ++i) a.ph[i] = R(p.ph[i]);
  if (a.sm.count == 0) return QD_OK;
  const int bs = tune().diag_block;
  hipLaunchKernelGGL((k_diag<R, 2>), dim3(grid_for(a.sm.count, uint64_t(bs) * 2)), dim3(bs), 0, s->stream, a);
  g_last_kernel = label<kKnDiag, R>();
  return check_launch("k_diag");
}

template <typename R>
static int launch_generic(qd_state* s, const GatePlan& p) {
  const Register& r = s->reg;
  int role[QD_MAX_QUDITS] = {};
  for (int j = 0; j < p.k; ++j) role[p.targets[j]] = 1;
  for (int j = 0; j < p.m; ++j) role[p.controls[j]] = 1;
  int64_t base = 0;
  for (int j = 0; j < p.m; ++j) base += int64_t(p.cvals[j]) * r.strides[p.controls[j]];
  const size_t bytes = sizeof(GenericHead) + sizeof(int64_t) * p.dT + sizeof(R) * 2 * size_t(p.dT) * p.dT;
  std::vector<unsigned char> buf(bytes, 0);
  auto* h = reinterpret_cast<GenericHead*>(buf.data());
  fill_slicemap64(make_groups(r, role, nullptr, 0, r.n), base, &h->sm);
  h->dT = p.dT;
  h->nsw = std::max(1, 1024 / p.dT);
  target_offsets(r, p, reinterpret_cast<int64_t*>(buf.data() + sizeof(GenericHead)));
  R* U = reinterpret_cast<R*>(buf.data() + sizeof(GenericHead) + sizeof(int64_t) * p.dT);
  for (size_t i = 0; i < 2 * size_t(p.dT) * p.dT; ++i) U[i] = R(p.U[i]);
  if (h->sm.count == 0) return QD_OK;
  void* dev = nullptr;
  int rc = ring_push(s, buf.data(), bytes, &dev);
  if (rc) return rc;
  const uint64_t iters = (h->sm.count + h->nsw - 1) / h->nsw;
  const unsigned grid = unsigned(std::min<uint64_t>(iters, 65536));
  const size_t lds = size_t(h->nsw) * p.dT * sizeof(R) * 2;
  hipLaunchKernelGGL((k_dense_generic<R>), dim3(grid), dim3(256), lds, s->stream, reinterpret_cast<R*>(s->data),
                     static_cast<const unsigned char*>(dev));
  g_last_kernel = label<kKnGeneric, R>();
  return check_launch("k_dense_generic");
}

template <typename R>
static int launch_gemm(qd_state* s, const GatePlan& p);

template <typename R, int DT>
static int launch_direct_lu(qd_state* s, const GatePlan& p) {
  const Register& r = s->reg;
  int role[QD_MAX_QUDITS] = {};
  for (int j = 0; j < p.k; ++j) role[p.targets[j]] = 1;
  for (int j = 0; j < p.m; ++j) role[p.controls[j]] = 1;
  int64_t base = 0;
  for (int j = 0; j < p.m; ++j) base += int64_t(p.cvals[j]) * r.strides[p.controls[j]];
  const size_t bytes = sizeof(LuHead) + sizeof(R) * 2 * size_t(DT) * DT;
  std::vector<unsigned char> buf(bytes, 0);
  auto* h = reinterpret_cast<LuHead*>(buf.data());
  if (fill_slicemap(make_groups(r, role, nullptr, 0, r.n), base, &h->sm) != QD_OK) return launch_gemm<R>(s, p);
  target_offsets(r, p, h->toff);
  R* U = reinterpret_cast<R*>(buf.data() + sizeof(LuHead));
  for (size_t i = 0; i < 2 * size_t(DT) * DT; ++i) U[i] = R(p.U[i]);
  if (h->sm.count == 0) return QD_OK;
  void* dev = nullptr;
  int rc = ring_push(s, buf.data(), bytes, &dev);
  if (rc) return rc;
  hipLaunchKernelGGL((k_slices_direct_lu<R, DT>), dim3(grid_for(h->sm.count, 256)), dim3(256), 0, s->stream,
                     reinterpret_cast<R*>(s->data), static_cast<const unsigned char*>(dev));
  g_last_kernel = label<kKnLu, R, DT>();
  return check_launch("k_slices_direct_lu");
}

template <typename R>
static int launch_gemm(qd_state* s, const GatePlan& p) {
  const Register& r = s->reg;
  int role[QD_MAX_QUDITS] = {};
  for (int j = 0; j < p.k; ++j) role[p.targets[j]] = 1;
  for (int j = 0; j < p.m; ++j) role[p.controls[j]] = 1;
  int64_t base = 0;
  for (int j = 0; j < p.m; ++j) base += int64_t(p.cvals[j]) * r.strides[p.controls[j]];
  const int dT = p.dT, dP = (dT + 3) / 4 * 4, ns = (kGemmOut / dP) / 4 * 4;
  const size_t bytes = sizeof(GemmHead) + sizeof(int64_t) * size_t(dT) + sizeof(int32_t) * size_t(dP) +
                       sizeof(R) * 2 * size_t(dP) * dP;
  std::vector<unsigned char> buf(bytes, 0);
  auto* h = reinterpret_cast<GemmHead*>(buf.data());
  const std::vector<Group> groups = make_groups(r, role, nullptr, 0, r.n);
  if (fill_slicemap(groups, base, &h->sm) != QD_OK) return launch_generic<R>(s, p);
  h->nsm = make_magic32(uint32_t(ns));
  h->dpm = make_magic32(uint32_t(dP));
  h->dT = dT;
  h->dP = dP;
  h->ns = ns;
  int64_t* toff = reinterpret_cast<int64_t*>(buf.data() + sizeof(GemmHead));
  target_offsets(r, p, toff);
  int32_t* yord = reinterpret_cast<int32_t*>(buf.data() + sizeof(GemmHead) + sizeof(int64_t) * size_t(dT));
  for (int y = 0; y < dP; ++y) yord[y] = y;
  std::sort(yord, yord + dT, [&](int32_t a, int32_t b) { return toff[a] < toff[b]; });
  int64_t tmin = INT64_MAX;
  for (int j = 0; j < p.k; ++j) tmin = std::min<int64_t>(tmin, r.strides[p.targets[j]]);
  h->yfast = groups.empty() || tmin < groups[0].stride ? 1 : 0;   // groups[0]: the lowest free run
  R* U = reinterpret_cast<R*>(buf.data() + sizeof(GemmHead) + sizeof(int64_t) * size_t(dT) + sizeof(int32_t) * size_t(dP));
  for (int a = 0; a < dT; ++a)
    for (int c = 0; c < dT; ++c) {
      U[2 * (size_t(a) * dP + c)] = R(p.U[2 * (size_t(a) * dT + c)]);
      U[2 * (size_t(a) * dP + c) + 1] = R(p.U[2 * (size_t(a) * dT + c) + 1]);
    }
  if (h->sm.count == 0) return QD_OK;
  void* dev = nullptr;
  int rc = ring_push(s, buf.data(), bytes, &dev);
  if (rc) return rc;
  using C = typename CxT<R>::T;
  const size_t lds = size_t(dP) * ns * sizeof(C) + size_t(dP) * (dP + 1) * sizeof(C) + sizeof(int64_t) * size_t(ns + dT) +
                     sizeof(int32_t) * size_t(dP);
  auto k = k_dense_gemm<R>;
  QD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  int dev_id = 0, cus = 256, per_cu = 0;
  (void)hipGetDevice(&dev_id);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  const uint64_t ntiles = (uint64_t(h->sm.count) + ns - 1) / ns;
  const unsigned grid = unsigned(std::min<uint64_t>(ntiles, uint64_t(cus) * per_cu));
  hipLaunchKernelGGL(k, dim3(grid), dim3(256), lds, s->stream, reinterpret_cast<R*>(s->data),
                     static_cast<const unsigned char*>(dev));
  g_last_kernel = label<kKnGemm, R>();
  return check_launch("k_dense_gemm");
}

template <typename R>
static int launch_gate_t(qd_state* s, const GatePlan& p) {
  const int route = route_gate(s->reg, s->prec, p);
  if (route == QD_ROUTE_GENERIC) return launch_generic<R>(s, p);
  if (route == QD_ROUTE_GEMM) return launch_gemm<R>(s, p);
  if (route == QD_ROUTE_DIAG) return launch_diag<R>(s, p);
  // On the slice-per-thread kernel a monomial U up to d_T = 9 runs as a dense one: each thread then
  // issues all its loads before its stores, which measured faster than storing every output as soon
  // as its one input arrives (a ququart shift 607 -> 588 us on a 1.7 GB state; with a control below
  // one line 720 -> 575 us), and the zero entries add exact zeros.
  if (p.cls == QD_CLASS_MONOMIAL && !(route == QD_ROUTE_DIRECT && p.dT <= kMaxInlineDense)) {
    switch (p.dT) {
      case 2: return launch_mono_t<R, 2>(s, p);
      case 3: return launch_mono_t<R, 3>(s, p);
      case 4: return launch_mono_t<R, 4>(s, p);
      case 5: return launch_mono_t<R, 5>(s, p);
      case 6: return launch_mono_t<R, 6>(s, p);
      case 7: return launch_mono_t<R, 7>(s, p);
      case 8: return launch_mono_t<R, 8>(s, p);
      case 9: return launch_mono_t<R, 9>(s, p);
      case 12: return launch_mono_t<R, 12>(s, p);
      case 16: return launch_mono_t<R, 16>(s, p);
      default: break;
    }
  }
  switch (p.dT) {
    case 2: return launch_dense_t<R, 2>(s, p);
    case 3: return launch_dense_t<R, 3>(s, p);
    case 4: return launch_dense_t<R, 4>(s, p);
    case 5: return launch_dense_t<R, 5>(s, p);
    case 6: return launch_dense_t<R, 6>(s, p);
    case 7: return launch_dense_t<R, 7>(s, p);
    case 8: return launch_dense_t<R, 8>(s, p);
    case 9: return launch_dense_t<R, 9>(s, p);
    case 12: return launch_direct_lu<R, 12>(s, p);
    case 16: return launch_direct_lu<R, 16>(s, p);
    default: return launch_generic<R>(s, p);
  }
}

int launch_gate(qd_state* s, const GatePlan& p) {
  g_last_kernel = "";
  return s->prec == QD_C128 ? launch_gate_t<double>(s, p) : launch_gate_t<float>(s, p);
}

const char* last_kernel() { return g_last_kernel; }
void set_last_kernel(const char* name) { g_last_kernel = name; }

}  // namespace qd
