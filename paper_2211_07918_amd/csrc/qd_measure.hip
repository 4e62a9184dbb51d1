// Readout after the gates: shots of a computational-basis measurement of every qudit (Sec. 2.2;
// measure_all, Sec. 3.1), per-qudit outcome distributions, and the list of basis states that
// carry probability, which run() prints as kets (Sec. 3.6, Sec. 3.8, example of Sec. 3.9).
//
// Probabilities are FP64, p = re*re + im*im with both products rounded before the sum.
//
// Shots invert the cumulative distribution of the integer weights w = round(p 2^62): exact
// integer sums, so the outcome of a random word r is the same whatever order the GPU adds in.
// With W = sum w, t = floor(r W / 2^64) and the shot is the first x whose cumulative weight
// exceeds t. Three levels of sums locate it: chunks of 64 amplitudes (one wavefront), blocks of
// 128 chunks (exclusive prefixes inside the block), and exclusive offsets of the blocks. A shot
// is one wavefront: a 64-way search over block offsets, one ballot over the block's chunk
// prefixes, one wavefront scan of the chunk's 64 weights recomputed from the state.
//
// The support list (states with p > eps, ascending) uses the same three levels on indicator
// values, so every wavefront knows where its chunk's entries go.
//
// Marginals: the register is cut into rows of T = d_k ... d_{n-1} <= 4096 amplitudes (k as small as
// that allows): the low qudits k..n-1 vary inside a row, the high ones are constant along it. One pass sums
// every row (row totals) and every column over the rows a workgroup owns (column partials); the
// column sums give the low qudits' marginals, and the row totals, a probability vector over the
// high qudits, go through the same pass again. All sums run in a fixed order: repeated calls
// return identical bits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "qd_internal.h"
#include "qd_stream.h"

namespace qd {
namespace {

constexpr int kChunk = 64;            // amplitudes per chunk: one wavefront
constexpr int kBlockChunks = 128;     // chunks per block
constexpr double kWeightScale = 0x1p62;
constexpr double kMaxProb = 3.999;    // a larger p (or a NaN) cannot be weighted in 64 bits
constexpr uint32_t kMargRow = 4096;   // longest row of the marginal pass
constexpr uint32_t kMargGrid = 1024;  // workgroups of the marginal pass (column partials)
constexpr unsigned kWaveGrid = 1u << 20;   // workgroups of the wavefront-per-item kernels (at most)

template <typename R> struct CxM;
template <> struct CxM<double> { using T = double2; };
template <> struct CxM<float> { using T = float2; };

// two rounded products and a rounded sum: contraction into a fused multiply-add is switched off
template <typename C>
__device__ __forceinline__ double prob_exact(C a) {
#pragma clang fp contract(off)
  const double re = double(a.x), im = double(a.y);
  const double rr = re * re, ii = im * im;
  return rr + ii;
}

__device__ __forceinline__ uint64_t weight_of(double p) {
  return p < kMaxProb ? uint64_t(rint(p * kWeightScale)) : 0ull;
}

__device__ __forceinline__ uint64_t wave_inclusive_scan(uint64_t x, uint32_t l) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(x, d, 64);
    if (l >= uint32_t(d)) x += y;
  }
  return x;
}

// exact sum of the 64 lanes' values; *over = true when it does not fit in 64 bits
__device__ __forceinline__ uint64_t wave_sum_checked(uint64_t v, bool* over) {
  uint64_t lo = v & 0xFFFFFFFFull, hi = v >> 32;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    lo += __shfl_xor(lo, d, 64);
    hi += __shfl_xor(hi, d, 64);
  }
  const uint64_t hs = hi + (lo >> 32);
  *over = (hs >> 32) != 0;
  return (hs << 32) | (lo & 0xFFFFFFFFull);
}

enum { VAL_WEIGHT = 0, VAL_SUPPORT = 1 };

// chunk[c] = sum over the chunk's amplitudes of their value (weight, or p > eps); a wavefront
// takes four chunks per iteration so that four loads per lane are in flight
template <typename R, int V>
__global__ __launch_bounds__(256) void k_chunk_values(const R* psi_raw, uint64_t D, double eps, uint64_t* chunk,
                                                      uint32_t* flag) {
  using C = typename CxM<R>::T;
  constexpr int U = 4;
  const C* psi = reinterpret_cast<const C*>(psi_raw);
  const uint64_t nch = (D + kChunk - 1) / kChunk;
  const uint32_t l = threadIdx.x & 63;
  const uint64_t nwaves = (uint64_t(gridDim.x) * blockDim.x) >> 6;
  for (uint64_t c0 = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6; c0 < nch; c0 += nwaves * U) {
    C a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = (c0 + uint64_t(u) * nwaves) * kChunk + l;
      if (i < D) a[u] = ld_stream(psi + i);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t c = c0 + uint64_t(u) * nwaves;
      if (c >= nch) break;   // wave-uniform
      const uint64_t i = c * kChunk + l;
      uint64_t v = 0;
      bool bad = false;
      if (i < D) {
        const double p = prob_exact(a[u]);
        if (V == VAL_WEIGHT) {
          bad = !(p < kMaxProb);
          v = weight_of(p);
        } else {
          v = p > eps ? 1u : 0u;
        }
      }
      bool over = false;
      const uint64_t sum = wave_sum_checked(v, &over);
      if (bad) flag[0] = 1u;
      if (l == 0) {
        chunk[c] = sum;
        if (over) flag[0] = 1u;
      }
    }
  }
}

// per block of 128 chunks: chunk values -> exclusive prefixes inside the block (in place), and
// the block total
__global__ __launch_bounds__(256) void k_block_scan(uint64_t* chunk, uint64_t nch, uint64_t* blk, uint32_t* flag) {
  const uint64_t nb = (nch + kBlockChunks - 1) / kBlockChunks;
  const uint32_t l = threadIdx.x & 63;
  const uint64_t nwaves = (uint64_t(gridDim.x) * blockDim.x) >> 6;
  for (uint64_t b = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6; b < nb; b += nwaves) {
    const uint64_t c0 = b * kBlockChunks;
    const bool in0 = c0 + l < nch, in1 = c0 + 64 + l < nch;
    const uint64_t a0 = in0 ? chunk[c0 + l] : 0, a1 = in1 ? chunk[c0 + 64 + l] : 0;
    bool o0 = false, o1 = false;
    const uint64_t t0 = wave_sum_checked(a0, &o0), t1 = wave_sum_checked(a1, &o1);
    const uint64_t x0 = wave_inclusive_scan(a0, l), x1 = wave_inclusive_scan(a1, l) + t0;
    if (in0) chunk[c0 + l] = x0 - a0;
    if (in1) chunk[c0 + 64 + l] = x1 - a1;
    if (l == 0) {
      blk[b] = t0 + t1;
      if (o0 || o1 || t0 + t1 < t0) flag[0] = 1u;
    }
  }
}

// one workgroup: block totals -> exclusive block offsets (in place) and the grand total.
// Thread t owns a contiguous segment; segment sums are scanned by wavefronts, then across the 16
// wavefronts.
__global__ __launch_bounds__(1024) void k_top_scan(uint64_t* blk, uint64_t nb, uint64_t* total, uint32_t* flag) {
  __shared__ uint64_t wtot[16];
  __shared__ uint32_t s_over;
  const uint32_t t = threadIdx.x, w = t >> 6, l = t & 63;
  const uint64_t seg = (nb + 1023) / 1024;
  const uint64_t s0 = std::min<uint64_t>(nb, uint64_t(t) * seg), s1 = std::min<uint64_t>(nb, s0 + seg);
  if (t == 0) s_over = 0;
  uint64_t s = 0;
  bool over = false;
  for (uint64_t i = s0; i < s1; ++i) {
    const uint64_t n = s + blk[i];
    over |= n < s;
    s = n;
  }
  bool wover = false;
  const uint64_t ws = wave_sum_checked(s, &wover);
  const uint64_t incl = wave_inclusive_scan(s, l);
  if (l == 0) wtot[w] = ws;
  __syncthreads();
  if (over || wover) s_over = 1;
  if (t == 0) {
    uint64_t acc = 0;
    for (int k = 0; k < 16; ++k) {
      const uint64_t v = wtot[k];
      wtot[k] = acc;
      const uint64_t n = acc + v;
      if (n < acc) s_over = 1;
      acc = n;
    }
    total[0] = acc;
  }
  __syncthreads();
  uint64_t a = wtot[w] + (incl - s);
  for (uint64_t i = s0; i < s1; ++i) {
    const uint64_t v = blk[i];
    blk[i] = a;
    a += v;
  }
  __syncthreads();
  if (t == 0 && s_over) flag[0] = 1u;
}

// four shots per wavefront in lockstep, so their chains of dependent loads overlap
template <typename R>
__global__ __launch_bounds__(256) void k_sample_shots(const R* psi_raw, uint64_t D, const uint64_t* chunkx,
                                                      uint64_t nch, const uint64_t* boff, uint64_t nb,
                                                      const uint64_t* totalp, const uint64_t* rnd, uint64_t shots,
                                                      int64_t* out) {
  using C = typename CxM<R>::T;
  constexpr int S = 4;
  const C* psi = reinterpret_cast<const C*>(psi_raw);
  const uint32_t l = threadIdx.x & 63;
  const uint64_t W = totalp[0];
  const uint64_t nwaves = (uint64_t(gridDim.x) * blockDim.x) >> 6;
  for (uint64_t j0 = ((uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6) * S; j0 < shots; j0 += nwaves * S) {
    uint64_t t[S], lo[S], n[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
      const uint64_t j = j0 + k;
      t[k] = j < shots ? __umul64hi(rnd[j], W) : 0;   // 0 <= t < W
      lo[k] = 0;
      n[k] = nb;
    }
    // block: the last b with boff[b] <= t (boff[0] = 0, nondecreasing); range [lo, lo + n)
    bool more = nb > 1;
    while (more) {
      uint64_t step[S];
      bool ok[S];
#pragma unroll
      for (int k = 0; k < S; ++k) {
        step[k] = (n[k] + 63) / 64;
        const uint64_t off = uint64_t(l) * step[k];
        ok[k] = n[k] > 1 && off < n[k] && boff[lo[k] + off] <= t[k];
      }
      more = false;
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const uint64_t m = __ballot(ok[k]);
        if (n[k] > 1) {   // wave-uniform; lane 0 always holds: boff[lo] <= t
          const uint64_t q = uint64_t(63 - __clzll(m));
          lo[k] += q * step[k];
          n[k] = std::min<uint64_t>(step[k], n[k] - q * step[k]);
          more |= n[k] > 1;
        }
      }
    }
    // chunk: the last k with chunkx[b 128 + k] <= t - boff[b]
    uint64_t r1[S], c0[S], a0[S], a1[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
      r1[k] = t[k] - boff[lo[k]];
      c0[k] = lo[k] * kBlockChunks;
      a0[k] = c0[k] + l < nch ? chunkx[c0[k] + l] : ~0ull;
      a1[k] = c0[k] + 64 + l < nch ? chunkx[c0[k] + 64 + l] : ~0ull;
    }
    uint64_t c[S], r2[S];
    C amp[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
      const uint64_t m0 = __ballot(a0[k] <= r1[k]), m1 = __ballot(a1[k] <= r1[k]);
      const uint64_t kc = m1 ? uint64_t(64 + 63 - __clzll(m1)) : uint64_t(63 - __clzll(m0));
      c[k] = c0[k] + kc;
      r2[k] = r1[k] - chunkx[c[k]];
      const uint64_t i = c[k] * kChunk + l;
      if (i < D) amp[k] = psi[i];
    }
    // amplitude: the first lane whose inclusive weight exceeds r2
#pragma unroll
    for (int k = 0; k < S; ++k) {
      const uint64_t i = c[k] * kChunk + l;
      const uint64_t w = i < D ? weight_of(prob_exact(amp[k])) : 0;
      const uint64_t x = wave_inclusive_scan(w, l);
      const uint64_t m = __ballot(x > r2[k]);
      if (l == 0 && j0 + k < shots) out[j0 + k] = int64_t(c[k] * kChunk + uint64_t(__ffsll(static_cast<long long>(m)) - 1));
    }
  }
}

// support list: entry number pos of the ascending list holds amplitude x with p_x > eps
template <typename R>
__global__ __launch_bounds__(256) void k_support_write(const R* psi_raw, uint64_t D, double eps,
                                                       const uint64_t* chunkx, const uint64_t* boff, uint64_t max_out,
                                                       int64_t* idx, R* amps, double* probs) {
  using C = typename CxM<R>::T;
  const C* psi = reinterpret_cast<const C*>(psi_raw);
  const uint64_t nch = (D + kChunk - 1) / kChunk;
  const uint32_t l = threadIdx.x & 63;
  const uint64_t nwaves = (uint64_t(gridDim.x) * blockDim.x) >> 6;
  const uint64_t below = (l == 0) ? 0ull : (~0ull >> (64 - l));   // lanes before this one
  for (uint64_t c = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6; c < nch; c += nwaves) {
    const uint64_t i = c * kChunk + l;
    C a{};
    double p = 0.0;
    bool keep = false;
    if (i < D) {
      a = psi[i];
      p = prob_exact(a);
      keep = p > eps;
    }
    const uint64_t m = __ballot(keep);
    if (keep) {
      const uint64_t pos = boff[c / kBlockChunks] + chunkx[c] + uint64_t(__popcll(m & below));
      if (pos < max_out) {
        if (idx) idx[pos] = int64_t(i);
        if (amps) reinterpret_cast<C*>(amps)[pos] = a;
        if (probs) probs[pos] = p;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------ marginals
__device__ __forceinline__ double prob_in(const double2* p, uint64_t i) { return prob_exact(ld_stream(p + i)); }
__device__ __forceinline__ double prob_in(const float2* p, uint64_t i) { return prob_exact(ld_stream(p + i)); }
__device__ __forceinline__ double prob_in(const double* p, uint64_t i) { return p[i]; }

// rows of T entries: row totals as four wavefront partials rowp[4 row + w]; column partials
// colp[g T + j] = sum over the rows of workgroup g (rows g, g + G, ...) of entry j
template <typename In>
__global__ __launch_bounds__(256) void k_marg_rows(const In* in, uint32_t T, uint64_t R, double* colp, double* rowp) {
  constexpr int M = kMargRow / 256;
  const uint32_t t = threadIdx.x, w = t >> 6, l = t & 63;
  double acc[M];
#pragma unroll
  for (int m = 0; m < M; ++m) acc[m] = 0.0;
  for (uint64_t row = blockIdx.x; row < R; row += gridDim.x) {
    const uint64_t base = row * T;
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const uint32_t j = t + 256u * m;
      if (j < T) {
        const double v = prob_in(in, base + j);
        acc[m] += v;
        s += v;
      }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
    if (l == 0) rowp[row * 4 + w] = s;
  }
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const uint32_t j = t + 256u * m;
    if (j < T) colp[uint64_t(blockIdx.x) * T + j] = acc[m];
  }
}

// column sums over the G partials in two fixed-order stages: workgroup (x, y) takes 64 columns and
// the partials g = y, y + 8, ... (4 wavefronts interleaved), then 8 values per column
constexpr uint32_t kColSplit = 8;
__global__ __launch_bounds__(256) void k_marg_cols(const double* colp, uint32_t G, uint32_t T, double* part) {
  __shared__ double sh[4][64];
  const uint32_t l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t j = blockIdx.x * 64 + l, y = blockIdx.y;
  double s = 0.0;
  if (j < T)
    for (uint32_t g = y + kColSplit * w; g < G; g += kColSplit * 4) s += colp[uint64_t(g) * T + j];
  sh[w][l] = s;
  __syncthreads();
  if (w == 0 && j < T) part[uint64_t(y) * T + j] = ((sh[0][l] + sh[1][l]) + sh[2][l]) + sh[3][l];
}

__global__ __launch_bounds__(256) void k_marg_cols_final(const double* part, uint32_t T, double* colsum) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= T) return;
  double s = 0.0;
  for (uint32_t y = 0; y < kColSplit; ++y) s += part[uint64_t(y) * T + j];
  colsum[j] = s;
}

__global__ __launch_bounds__(256) void k_marg_rowsum(const double* rowp, uint64_t R, double* rowsum) {
  const uint64_t r = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r < R) rowsum[r] = ((rowp[4 * r] + rowp[4 * r + 1]) + rowp[4 * r + 2]) + rowp[4 * r + 3];
}

// marginals of the qudits that vary inside a row: pair (q, v) sums the column sums whose digit
// (j / stride) mod dim equals v, i.e. the columns a (dim stride) + v stride + b. One wavefront per
// pair: lane l takes every 64th such column, then a fixed butterfly adds the lanes.
struct LowQudits {
  int32_t nq;
  int32_t dim[QD_MAX_QUDITS];
  int32_t stride[QD_MAX_QUDITS];   // inside the row (< 4096)
  int32_t out_off[QD_MAX_QUDITS];  // where the qudit's d values go
  int32_t npairs;
};

__global__ __launch_bounds__(256) void k_marg_low(const double* colsum, uint32_t T, LowQudits lq, double* out) {
  const int p = int((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const uint32_t l = threadIdx.x & 63;
  if (p >= lq.npairs) return;   // wave-uniform
  int q = 0, v = p;
  while (v >= lq.dim[q]) {
    v -= lq.dim[q];
    ++q;
  }
  const uint32_t d = uint32_t(lq.dim[q]), st = uint32_t(lq.stride[q]);
  const uint32_t cnt = T / d;   // columns with this digit: (T / (d st)) runs of st
  double s = 0.0;
  for (uint32_t e = l; e < cnt; e += 64) {
    const uint32_t a = e / st, b = e - a * st;
    s += colsum[a * d * st + uint32_t(v) * st + b];
  }
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) s += __shfl_xor(s, k, 64);
  if (l == 0) out[lq.out_off[q] + v] = s;
}

// ------------------------------------------------------------------------------------------ host side
struct MeasureWs {
  uint64_t* chunk = nullptr;
  uint64_t* blk = nullptr;
  uint64_t* total = nullptr;
  uint32_t* flag = nullptr;
  uint64_t nch = 0, nb = 0;
};

int ensure_ws(qd_state* s, size_t bytes, bool* moved = nullptr) {
  if (moved) *moved = false;
  if (s->mws_cap >= bytes) return QD_OK;
  if (moved) *moved = true;
  if (s->mws) {
    (void)hipStreamSynchronize(s->stream);
    (void)hipFree(s->mws);
  }
  s->mws = nullptr;
  s->mws_cap = 0;
  QD_HIP(hipMalloc(&s->mws, bytes));
  s->mws_cap = bytes;
  return QD_OK;
}

unsigned wave_grid(uint64_t items) {
  return unsigned(std::max<uint64_t>(1, std::min<uint64_t>((items + 3) / 4, kWaveGrid)));
}

// the three levels of sums of per-amplitude values; `extra` bytes of workspace follow them
template <typename R>
int scan_values(qd_state* s, int v, double eps, size_t extra, MeasureWs* w, size_t* extra_off) {
  const uint64_t D = uint64_t(s->reg.D);
  w->nch = (D + kChunk - 1) / kChunk;
  w->nb = (w->nch + kBlockChunks - 1) / kBlockChunks;
  const size_t head = (w->nch + w->nb + 2) * sizeof(uint64_t);
  const size_t off = (head + 255) & ~size_t(255);
  int rc = ensure_ws(s, off + extra);
  if (rc) return rc;
  w->chunk = reinterpret_cast<uint64_t*>(s->mws);
  w->blk = w->chunk + w->nch;
  w->total = w->blk + w->nb;
  w->flag = reinterpret_cast<uint32_t*>(w->total + 1);
  *extra_off = off;
  QD_HIP(hipMemsetAsync(w->flag, 0, sizeof(uint64_t), s->stream));
  const R* psi = reinterpret_cast<const R*>(s->data);
  if (v == VAL_WEIGHT)
    hipLaunchKernelGGL((k_chunk_values<R, VAL_WEIGHT>), dim3(wave_grid((w->nch + 3) / 4)), dim3(256), 0, s->stream, psi, D, eps,
                       w->chunk, w->flag);
  else
    hipLaunchKernelGGL((k_chunk_values<R, VAL_SUPPORT>), dim3(wave_grid((w->nch + 3) / 4)), dim3(256), 0, s->stream, psi, D, eps,
                       w->chunk, w->flag);
  QD_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_block_scan, dim3(wave_grid(w->nb)), dim3(256), 0, s->stream, w->chunk, w->nch, w->blk, w->flag);
  QD_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_top_scan, dim3(1), dim3(1024), 0, s->stream, w->blk, w->nb, w->total, w->flag);
  QD_HIP(hipGetLastError());
  return QD_OK;
}

// total and flag to the host (synchronises)
int read_total(qd_state* s, const MeasureWs& w, uint64_t* total, uint32_t* flag) {
  uint64_t buf[2];
  QD_HIP(hipMemcpyAsync(buf, w.total, sizeof(buf), hipMemcpyDeviceToHost, s->stream));
  QD_HIP(hipStreamSynchronize(s->stream));
  *total = buf[0];
  *flag = uint32_t(buf[1] & 0xFFFFFFFFull);
  return QD_OK;
}

template <typename R>
int sample_t(qd_state* s, const uint64_t* rand, int64_t shots, int64_t* out, int on_device) {
  MeasureWs w;
  size_t off = 0;
  const size_t stage = on_device ? 0 : size_t(shots) * (sizeof(uint64_t) + sizeof(int64_t));
  int rc = scan_values<R>(s, VAL_WEIGHT, 0.0, stage, &w, &off);
  if (rc) return rc;
  uint64_t total = 0;
  uint32_t flag = 0;
  rc = read_total(s, w, &total, &flag);
  if (rc) return rc;
  if (flag) return fail(QD_EINVAL, "state too far from unit norm to sample (squared norm must stay below 3.999)");
  if (total == 0) return fail(QD_EINVAL, "state has no probability to sample");
  const uint64_t* d_rand = rand;
  int64_t* d_out = out;
  if (!on_device) {
    uint64_t* r = reinterpret_cast<uint64_t*>(static_cast<char*>(s->mws) + off);
    d_rand = r;
    d_out = reinterpret_cast<int64_t*>(r + shots);
    QD_HIP(hipMemcpyAsync(r, rand, size_t(shots) * sizeof(uint64_t), hipMemcpyHostToDevice, s->stream));
  }
  hipLaunchKernelGGL((k_sample_shots<R>), dim3(wave_grid((uint64_t(shots) + 3) / 4)), dim3(256), 0, s->stream,
                     reinterpret_cast<const R*>(s->data), uint64_t(s->reg.D), w.chunk, w.nch, w.blk, w.nb, w.total,
                     d_rand, uint64_t(shots), d_out);
  QD_HIP(hipGetLastError());
  if (!on_device)
    QD_HIP(hipMemcpyAsync(out, d_out, size_t(shots) * sizeof(int64_t), hipMemcpyDeviceToHost, s->stream));
  QD_HIP(hipStreamSynchronize(s->stream));
  return QD_OK;
}

template <typename R>
int support_t(qd_state* s, double eps, int64_t max_out, int64_t* idx, void* amps, double* probs, int64_t* count) {
  MeasureWs w;
  size_t off = 0;
  int rc = scan_values<R>(s, VAL_SUPPORT, eps, 0, &w, &off);
  if (rc) return rc;
  uint64_t total = 0;
  uint32_t flag = 0;
  rc = read_total(s, w, &total, &flag);
  if (rc) return rc;
  if (count) *count = int64_t(total);
  const uint64_t nout = std::min<uint64_t>(total, uint64_t(std::max<int64_t>(max_out, 0)));
  if (nout == 0 || (!idx && !amps && !probs)) return QD_OK;
  const size_t per = sizeof(int64_t) + 2 * sizeof(R) + sizeof(double);
  bool moved = false;
  rc = ensure_ws(s, off + nout * per, &moved);
  if (rc) return rc;
  if (moved) {   // the larger workspace lost the sums: run the three levels again
    rc = scan_values<R>(s, VAL_SUPPORT, eps, nout * per, &w, &off);
    if (rc) return rc;
  }
  char* base = static_cast<char*>(s->mws) + off;
  int64_t* d_idx = reinterpret_cast<int64_t*>(base);
  double* d_prob = reinterpret_cast<double*>(d_idx + nout);
  R* d_amp = reinterpret_cast<R*>(d_prob + nout);
  hipLaunchKernelGGL((k_support_write<R>), dim3(wave_grid(w.nch)), dim3(256), 0, s->stream,
                     reinterpret_cast<const R*>(s->data), uint64_t(s->reg.D), eps, w.chunk, w.blk, nout,
                     idx ? d_idx : nullptr, amps ? d_amp : nullptr, probs ? d_prob : nullptr);
  QD_HIP(hipGetLastError());
  if (idx) QD_HIP(hipMemcpyAsync(idx, d_idx, nout * sizeof(int64_t), hipMemcpyDeviceToHost, s->stream));
  if (probs) QD_HIP(hipMemcpyAsync(probs, d_prob, nout * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  if (amps) QD_HIP(hipMemcpyAsync(amps, d_amp, nout * 2 * sizeof(R), hipMemcpyDeviceToHost, s->stream));
  QD_HIP(hipStreamSynchronize(s->stream));
  return QD_OK;
}

// one marginal level over a register (dims, n) whose entries are `in` (complex state or FP64)
template <typename In>
int marg_level(qd_state* s, const In* in, const int32_t* dims, int n, int32_t out_first, double* out_dev,
               double* colp, double* rowp, double* colsum, double* colpart, double* rows_a, double* rows_b) {
  int64_t st[QD_MAX_QUDITS];
  int64_t acc = 1;
  for (int q = n - 1; q >= 0; --q) {
    st[q] = acc;
    acc *= dims[q];
  }
  const uint64_t D = uint64_t(acc);
  // low qudits k..n-1: the longest suffix whose product fits in a row
  int k = n - 1;
  while (k > 0 && uint64_t(st[k - 1]) * uint64_t(dims[k - 1]) <= kMargRow) --k;
  const uint32_t T = uint32_t(st[k] * dims[k]);
  const int k_low = k;
  const uint64_t R = D / T;
  const uint32_t G = uint32_t(std::min<uint64_t>(R, kMargGrid));
  hipLaunchKernelGGL((k_marg_rows<In>), dim3(G), dim3(256), 0, s->stream, in, T, R, colp, rowp);
  QD_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_marg_cols, dim3((T + 63) / 64, kColSplit), dim3(256), 0, s->stream, colp, G, T, colpart);
  QD_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_marg_cols_final, dim3((T + 255) / 256), dim3(256), 0, s->stream, colpart, T, colsum);
  QD_HIP(hipGetLastError());
  LowQudits lq{};
  lq.nq = n - k_low;
  int32_t o = 0;
  for (int q = 0; q < k_low; ++q) o += dims[q];
  int pairs = 0;
  for (int q = k_low; q < n; ++q) {
    lq.dim[q - k_low] = dims[q];
    lq.stride[q - k_low] = int32_t(st[q]);
    lq.out_off[q - k_low] = out_first + o;
    o += dims[q];
    pairs += dims[q];
  }
  lq.npairs = pairs;
  hipLaunchKernelGGL(k_marg_low, dim3((pairs + 3) / 4), dim3(256), 0, s->stream, colsum, T, lq, out_dev);
  QD_HIP(hipGetLastError());
  if (k_low == 0) return QD_OK;
  hipLaunchKernelGGL(k_marg_rowsum, dim3(unsigned((R + 255) / 256)), dim3(256), 0, s->stream, rowp, R, rows_a);
  QD_HIP(hipGetLastError());
  // the row totals are a probability vector over qudits 0..k_low-1
  return marg_level<double>(s, rows_a, dims, k_low, out_first, out_dev, colp, rowp, colsum, colpart, rows_b, rows_a);
}

template <typename R>
int marginals_t(qd_state* s, double* out) {
  const Register& r = s->reg;
  int32_t nout = 0;
  for (int q = 0; q < r.n; ++q) nout += r.dims[q];
  // rows of the first level; later levels have fewer rows, and every level's column partials fit
  // in kMargGrid x kMargRow doubles
  int k = r.n - 1;
  while (k > 0 && uint64_t(r.strides[k - 1]) * uint64_t(r.dims[k - 1]) <= kMargRow) --k;
  const uint64_t R0 = uint64_t(r.D) / (uint64_t(r.strides[k]) * uint64_t(r.dims[k]));
  const size_t ncolp = size_t(kMargGrid) * kMargRow;
  const size_t doubles = ncolp + 4 * R0 + kMargRow * (1 + kColSplit) + 2 * R0 + size_t(nout);
  int rc = ensure_ws(s, doubles * sizeof(double));
  if (rc) return rc;
  double* colp = reinterpret_cast<double*>(s->mws);
  double* rowp = colp + ncolp;
  double* colsum = rowp + 4 * R0;
  double* colpart = colsum + kMargRow;
  double* rows_a = colpart + size_t(kColSplit) * kMargRow;
  double* rows_b = rows_a + R0;
  double* out_dev = rows_b + R0;
  using C = typename CxM<R>::T;
  rc = marg_level<C>(s, reinterpret_cast<const C*>(s->data), r.dims, r.n, 0, out_dev, colp, rowp, colsum, colpart,
                     rows_a, rows_b);
  if (rc) return rc;
  QD_HIP(hipMemcpyAsync(out, out_dev, size_t(nout) * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  QD_HIP(hipStreamSynchronize(s->stream));
  return QD_OK;
}

}  // namespace
}  // namespace qd

using namespace qd;

extern "C" {

int qd_sample(qd_state* s, const uint64_t* rand, int64_t shots, int64_t* out, int32_t on_device) {
  if (!s) return fail(QD_EINVAL, "null state");
  if (shots < 0) return fail(QD_EINVAL, "negative shot count");
  if (shots == 0) return QD_OK;
  if (!rand || !out) return fail(QD_EINVAL, "null random words or output");
  QD_HIP(hipSetDevice(s->device));
  return s->prec == QD_C128 ? sample_t<double>(s, rand, shots, out, on_device)
                            : sample_t<float>(s, rand, shots, out, on_device);
}

int qd_support(qd_state* s, double eps, int64_t max_out, int64_t* idx, void* amps, double* probs, int64_t* count) {
  if (!s) return fail(QD_EINVAL, "null state");
  if (!(eps >= 0.0)) return fail(QD_EINVAL, "eps must be >= 0");
  QD_HIP(hipSetDevice(s->device));
  return s->prec == QD_C128 ? support_t<double>(s, eps, max_out, idx, amps, probs, count)
                            : support_t<float>(s, eps, max_out, idx, amps, probs, count);
}

int qd_marginals(qd_state* s, double* out) {
  if (!s) return fail(QD_EINVAL, "null state");
  if (!out) return fail(QD_EINVAL, "null output");
  QD_HIP(hipSetDevice(s->device));
  return s->prec == QD_C128 ? marginals_t<double>(s, out) : marginals_t<float>(s, out);
}

int qd_ket_string(const int32_t* dims, int32_t n, int64_t index, char* buf, int32_t buflen) {
  if (!dims || n < 1 || n > QD_MAX_QUDITS) return fail(QD_EDIM, "bad register");
  if (!buf || buflen < 1) return fail(QD_EINVAL, "null or empty buffer");
  int64_t D = 1;
  int32_t dmax = 0;
  for (int q = 0; q < n; ++q) {
    if (dims[q] < 2 || dims[q] > QD_MAX_RADIX) return fail(QD_EDIM, "qudit dimension must be 2..256");
    D *= dims[q];
    dmax = std::max(dmax, dims[q]);
  }
  if (index < 0 || index >= D) return fail(QD_EINVAL, "index outside the register");
  std::vector<int32_t> dig(static_cast<size_t>(n), 0);
  int64_t rem = index;
  for (int q = n - 1; q >= 0; --q) {
    dig[size_t(q)] = int32_t(rem % dims[q]);
    rem /= dims[q];
  }
  std::string sres = "|";
  for (int q = 0; q < n; ++q) {
    if (q && dmax > 10) sres += ",";
    sres += std::to_string(dig[size_t(q)]);
  }
  sres += ">";
  if (int32_t(sres.size()) + 1 > buflen) return fail(QD_EINVAL, "buffer too small for the ket");
  std::memcpy(buf, sres.c_str(), sres.size() + 1);
  return QD_OK;
}

}  // extern "C"
