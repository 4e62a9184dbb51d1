// Sparse state: the list of a state's non-zero amplitudes with their flat indices, updated gate by
// gate on the GPU. It is the compressed sparse column of Sec. 3.3 (only non-zero amplitudes and
// their indices are stored) and the SparseBackend of Sec. 3.7 (operator products skip zero
// elements), applied gate by gate instead of through Kronecker-product operators.
//
// Rules (stated with the API in qd.h):
//   * an index is present exactly when its amplitude is not exactly zero: a dense-gate output whose
//     two parts are 0.0 is dropped; entries moved by a monomial gate are kept;
//   * a monomial gate (one non-zero entry in every row and column: shifts, generalized CNOTs, Z_d,
//     controlled phases, qudit swaps) moves each matching entry where it stands: its index gains
//     delta[loc] and its amplitude is multiplied by the column's entry unless that entry is exactly
//     1. The count does not change and the host does not wait;
//   * any other gate is dense: matching entries that share every non-target digit form a slice and
//     the slice's d_T outputs are U times its d_T inputs (absent inputs are zero). A product is
//     (ur xr - ui xi, ur xi + ui xr) and a sum runs over columns 0..d_T-1 from +0.0, every real
//     operation rounded on its own (no contraction into fused multiply-adds), so every bit of the
//     result, and so every drop decision, is fixed;
//   * list order: a monomial gate keeps every position; a dense gate keeps the non-matching entries
//     in their order and writes each slice's non-zero outputs, by increasing local row, where the
//     slice's first entry stood.
//
// HBM layout: two list buffers (int64 idx[cap], double2 amp[cap]); a dense gate reads one and
// writes the other. Device counters hold each buffer's entry count, so no launch needs the count
// on the host. A dense gate uses an open-addressing table of slice keys (linear probing with a
// 64-bit compare-and-swap), the first list position per key (atomic minimum), a reduce-then-scan
// that ranks slices by that position, a gather buffer of ns x d_T inputs and an output buffer of
// the same size, and a second reduce-then-scan that places the outputs. It waits once on the
// host, for ns, to size the gather buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "qd_internal.h"

// ------------------------------------------------------------------------------------------ types
namespace qd {
namespace sp {

// n / d for n < 2^63 by one 64-bit multiply-high (Granlund and Montgomery, PLDI 1994, Thm. 4.2
// with N = 63): l = ceil(log2 d), mul = ceil(2^(63+l) / d) < 2^64, n / d = mulhi(mul, n) >> (l-1).
// d = 1 is flagged and returns n.
struct Magic64 {
  uint64_t mul;
  uint32_t sh;
  uint32_t one;
};

static Magic64 make_magic64(uint64_t d) {
  Magic64 m{};
  if (d == 1) {
    m.one = 1;
    return m;
  }
  uint32_t l = 0;
  while (l < 63 && (uint64_t(1) << l) < d) ++l;
  if ((uint64_t(1) << l) < d) l = 64;                  // d > 2^63 (not reached: strides < 2^63)
  const unsigned __int128 num = (unsigned __int128)1 << (63 + l);
  m.mul = uint64_t((num + d - 1) / d);
  m.sh = l - 1;
  return m;
}

struct Qudit {
  Magic64 ms;      // division by the qudit's stride
  Magic64 md;      // division by its dimension
  uint32_t d;
  int32_t v;       // control value (controls only)
};

// targets first (first listed target most significant in the local index), then controls
struct Desc {
  uint32_t k, m, dT, pad;
  Qudit q[QD_MAX_QUDITS];
};

constexpr int kBlock = 256;
constexpr int kRounds = 8;
constexpr int64_t kChunk = int64_t(kBlock) * kRounds;   // list positions per scan block
constexpr uint64_t kEmpty = ~uint64_t(0);
constexpr int64_t kMaxEntries = int64_t(INT32_MAX);      // positions are int32 in the key table

// misc device words: [0], [1] entry counts of list buffers 0 and 1; [2] slices of the running
// dense gate; [3] key-table overflow flag; [8 ..] entries written by gates so far, spread over
// kUpdSlots counters (workgroup b adds to slot b mod kUpdSlots) so that no address takes more than
// a small share of the atomics
constexpr int kUpdSlots = 256;
enum { kCnt0 = 0, kNs = 2, kErr = 3, kUpd = 8, kMisc = 8 + kUpdSlots };

struct DevBuf {   // device buffer with its capacity in elements
  void* p = nullptr;
  size_t cap = 0;
};

}  // namespace sp
}  // namespace qd

struct qd_sparse {
  qd::Register reg;
  hipStream_t stream = nullptr;
  int device = 0;
  int64_t cap = 0;                  // entries per list buffer
  int64_t* idx[2] = {nullptr, nullptr};
  double2* amp[2] = {nullptr, nullptr};
  int cur = 0;
  int64_t bound = 0;                // upper bound on the current count
  int64_t* misc = nullptr;          // device words (see kCnt0..)
  int64_t* hmisc = nullptr;         // pinned host mirror
  qd::ParamRing ring;
  // dense-gate workspace: key table (keys, first position, slice rank per slot), per-entry slot
  // and local index, chunk sums, gathered inputs and outputs
  qd::sp::DevBuf keys, first, sid, slot_of, loc_of, bsum, xbuf, ybuf;
};

namespace qd {
namespace sp {

// ------------------------------------------------------------------------------------------ device helpers
__device__ __forceinline__ uint64_t mdiv(uint64_t n, const Magic64& m) {
  return m.one ? n : (__umul64hi(m.mul, n) >> m.sh);
}

__device__ __forceinline__ uint32_t digit(uint64_t x, const Qudit& q) {
  const uint64_t t = mdiv(x, q.ms);
  return uint32_t(t - mdiv(t, q.md) * q.d);
}

// control digits match -> true, with the local column index of the target digits
__device__ __forceinline__ bool analyse(uint64_t x, const Desc* __restrict__ g, uint32_t& loc) {
  const uint32_t k = g->k, m = g->m;
  for (uint32_t j = 0; j < m; ++j)
    if (digit(x, g->q[k + j]) != uint32_t(g->q[k + j].v)) return false;
  uint32_t l = 0;
  for (uint32_t j = 0; j < k; ++j) l = l * g->q[j].d + digit(x, g->q[j]);
  loc = l;
  return true;
}

// u * x with every real operation rounded on its own
__device__ __forceinline__ double2 cmul(double2 u, double2 x) {
#pragma clang fp contract(off)
  const double a = u.x * x.x;
  const double b = u.y * x.y;
  const double c = u.x * x.y;
  const double e = u.y * x.x;
  return make_double2(a - b, c + e);
}

__device__ __forceinline__ bool nonzero(double2 a) { return a.x != 0.0 || a.y != 0.0; }

// inclusive scan over a 64-lane wavefront
__device__ __forceinline__ int wave_incl(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// add the wavefront's sum of v to this workgroup's update counter (one atomic per wavefront)
__device__ __forceinline__ void wave_count(int v, int64_t* counters) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0 && v)
    atomicAdd(reinterpret_cast<unsigned long long*>(counters + (blockIdx.x & (kUpdSlots - 1))), (unsigned long long)v);
}

// exclusive scan of one value per thread over the 256-thread block; *total gets the block sum
__device__ __forceinline__ int block_excl(int v, int* sh, int* total) {
  const int incl = wave_incl(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) sh[w] = incl;
  __syncthreads();
  int off = 0;
#pragma unroll
  for (int i = 0; i < kBlock / 64; ++i) off += i < w ? sh[i] : 0;
  *total = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return off + incl - v;
}

// ------------------------------------------------------------------------------------------ monomial gates
constexpr int kMonoE = 4;            // entries per thread: all their loads are issued first
constexpr int kMonoTab = 1024;       // largest d_T, so the tables fit LDS

// UNIT: every column's entry is exactly 1, so amplitudes are neither read nor written. Entry e of
// workgroup b is b * kMonoE * kBlock + j * kBlock + lane (j < kMonoE): each load instruction reads
// a contiguous run of the list.
template <bool UNIT>
__global__ __launch_bounds__(kBlock) void k_monomial(const int64_t* __restrict__ cnt, int64_t* __restrict__ idx,
                                                     double2* __restrict__ amp, const Desc* __restrict__ g,
                                                     const int64_t* __restrict__ delta, const double2* __restrict__ ph,
                                                     const uint8_t* __restrict__ unit, int64_t* __restrict__ upd) {
  __shared__ int64_t s_delta[kMonoTab];
  __shared__ double2 s_ph[UNIT ? 1 : kMonoTab];
  __shared__ uint8_t s_unit[UNIT ? 1 : kMonoTab];
  const uint32_t k = g->k, m = g->m, dT = g->dT;
  for (uint32_t c = threadIdx.x; c < dT; c += kBlock) {
    s_delta[c] = delta[c];
    if (!UNIT) {
      s_ph[c] = ph[c];
      s_unit[c] = unit[c];
    }
  }
  const int64_t n = *cnt;
  const int64_t base = int64_t(blockIdx.x) * (kMonoE * kBlock) + threadIdx.x;
  uint64_t x[kMonoE];
  bool ok[kMonoE];
  uint32_t loc[kMonoE];
#pragma unroll
  for (int e = 0; e < kMonoE; ++e) {
    const int64_t pos = base + int64_t(e) * kBlock;
    ok[e] = pos < n;
    x[e] = ok[e] ? uint64_t(__builtin_nontemporal_load(idx + pos)) : 0;
    loc[e] = 0;
  }
  for (uint32_t j = 0; j < m; ++j) {
    const Qudit q = g->q[k + j];
#pragma unroll
    for (int e = 0; e < kMonoE; ++e) ok[e] = ok[e] && digit(x[e], q) == uint32_t(q.v);
  }
  for (uint32_t j = 0; j < k; ++j) {
    const Qudit q = g->q[j];
#pragma unroll
    for (int e = 0; e < kMonoE; ++e) loc[e] = loc[e] * q.d + digit(x[e], q);
  }
  __syncthreads();                   // tables staged
  int hits = 0;
#pragma unroll
  for (int e = 0; e < kMonoE; ++e) {
    if (ok[e]) {
      const int64_t pos = base + int64_t(e) * kBlock;
      __builtin_nontemporal_store(int64_t(x[e]) + s_delta[loc[e]], idx + pos);
      if (!UNIT && !s_unit[loc[e]]) amp[pos] = cmul(s_ph[loc[e]], amp[pos]);
      ++hits;
    }
  }
  wave_count(hits, upd);
}

// ------------------------------------------------------------------------------------------ fused runs
// A run of monomial gates applied in one pass: each entry's digits are decoded once into LDS (one
// byte per qudit), every gate of the run updates them (a shift X_{+a} adds a mod d; a table gate
// replaces its target digits by those of the row its column maps to and multiplies the amplitude),
// and the index is encoded and written once. Per entry the operations and their order are those of
// the gate-by-gate path, so the results are the same bits. The run's gate descriptors and tables
// (at most kRunStage bytes per launch) are staged in LDS once per workgroup and read by broadcast;
// workgroups are persistent and walk the list.
constexpr int kRunK = 4;             // targets per gate in a fused run
constexpr int kRunM = 8;             // controls per gate in a fused run
constexpr int kRunMin = 4;           // shorter runs go gate by gate
constexpr int kRunStage = 8192;      // bytes of descriptors and tables per launch
constexpr int kRunBlocksPerCU = 8;

struct RunGateC {                    // 32 bytes
  uint8_t shift, k, m, pad;          // shift > 0: X_{+shift} on one target with unit entries
  uint8_t tq[kRunK];                 // targets, first most significant
  uint8_t td1[kRunK];                // their dimensions minus one
  uint8_t cq[kRunM];                 // controls
  uint8_t cv[kRunM];                 // control values
  int32_t tab;                       // first table row of a table gate
};
static_assert(sizeof(RunGateC) == 32, "descriptor layout");

struct RunQudit {
  Magic64 md;                        // division by the qudit's dimension
  int64_t stride;
  uint32_t d, pad;
};

__device__ __forceinline__ uint32_t byte_of(uint32_t w, int i) { return (w >> (8 * i)) & 0xffu; }

// Each thread carries E entries; entry i's digit of qudit q sits at dig[(q * E + i) * kBlock + lane].
// Gate descriptors are read from device memory with scalar loads (uniform), one gate ahead; the
// tables of table gates are staged in LDS and read per lane.
template <int E>
__device__ __forceinline__ void control_check(const uint8_t* my, uint32_t cq, uint32_t cv, bool (&ok)[E]) {
  constexpr int QS = E * kBlock;
#pragma unroll
  for (int i = 0; i < E; ++i) ok[i] = ok[i] & (uint32_t(my[cq * QS + i * kBlock]) == cv);
}

template <bool UNIT, int kRunE>
__global__ __launch_bounds__(kBlock) void k_mono_run(const int64_t* __restrict__ cnt, int64_t* __restrict__ idx,
                                                     double2* __restrict__ amp, const uint4* __restrict__ stage,
                                                     int32_t stage16, int32_t ngates, int32_t o_nd, int32_t o_ph,
                                                     int32_t o_un, const RunQudit* __restrict__ rq, int32_t nq,
                                                     int64_t* __restrict__ upd) {
  extern __shared__ uint4 lds[];
  // tables only (the descriptors are read from device memory below)
  const int32_t t16 = (o_nd / 16);
  for (int i = t16 + int(threadIdx.x); i < stage16; i += kBlock) lds[i] = stage[i];
  const uint8_t* stg = reinterpret_cast<const uint8_t*>(lds);
  const uint32_t* nd = reinterpret_cast<const uint32_t*>(stg + o_nd);
  const double2* ph = reinterpret_cast<const double2*>(stg + o_ph);
  const uint8_t* un = stg + o_un;
  const uint4* gdesc = stage;                                          // two uint4 per gate
  uint8_t* my = reinterpret_cast<uint8_t*>(lds + stage16) + threadIdx.x;
  constexpr int QS = kRunE * kBlock;                                   // stride between qudits
  __syncthreads();
  const int64_t n = *cnt;
  uint32_t hits = 0;                                                   // uniform: counted by ballots
  for (int64_t b0 = int64_t(blockIdx.x) * (kRunE * kBlock); b0 < n; b0 += int64_t(gridDim.x) * (kRunE * kBlock)) {
    int64_t e[kRunE];
    bool active[kRunE];
    uint64_t x0[kRunE];
#pragma unroll
    for (int i = 0; i < kRunE; ++i) {
      e[i] = b0 + i * kBlock + threadIdx.x;
      active[i] = e[i] < n;
      x0[i] = active[i] ? uint64_t(__builtin_nontemporal_load(idx + e[i])) : 0;
    }
    {
      uint64_t t[kRunE];
#pragma unroll
      for (int i = 0; i < kRunE; ++i) t[i] = x0[i];
      for (int q = nq - 1; q >= 0; --q) {
        const RunQudit r = rq[q];
#pragma unroll
        for (int i = 0; i < kRunE; ++i) {
          const uint64_t qt = mdiv(t[i], r.md);
          my[q * QS + i * kBlock] = uint8_t(t[i] - qt * r.d);
          t[i] = qt;
        }
      }
    }
    double2 a[kRunE];
    bool changed[kRunE];
#pragma unroll
    for (int i = 0; i < kRunE; ++i) {
      a[i] = make_double2(0.0, 0.0);
      if (!UNIT && active[i]) a[i] = amp[e[i]];
      changed[i] = false;
    }
    for (int gi = 0; gi < ngates; ++gi) {
      const uint4 A = gdesc[2 * gi], B = gdesc[2 * gi + 1];           // scalar loads (uniform address)
      const uint32_t w0 = A.x, m = byte_of(w0, 2), shift = byte_of(w0, 0);
      bool ok[kRunE];
#pragma unroll
      for (int i = 0; i < kRunE; ++i) ok[i] = active[i];
      if (m >= 1) control_check<kRunE>(my, byte_of(A.w, 0), byte_of(B.y, 0), ok);
      if (m >= 2) control_check<kRunE>(my, byte_of(A.w, 1), byte_of(B.y, 1), ok);
      for (uint32_t j = 2; j < m; ++j)
        control_check<kRunE>(my, byte_of(j < 4 ? A.w : B.x, int(j & 3)), byte_of(j < 4 ? B.y : B.z, int(j & 3)), ok);
#pragma unroll
      for (int i = 0; i < kRunE; ++i) hits += uint32_t(__popcll(__ballot(ok[i])));
      if (shift) {
        const uint32_t q = byte_of(A.y, 0), d = byte_of(A.z, 0) + 1;
#pragma unroll
        for (int i = 0; i < kRunE; ++i) {
          if (ok[i]) {
            uint8_t* dq = my + q * QS + i * kBlock;
            const uint32_t v = uint32_t(*dq) + shift;
            *dq = uint8_t(v >= d ? v - d : v);
          }
        }
      } else {
        const uint32_t k = byte_of(w0, 1);
        const int32_t tab = int32_t(B.w);
#pragma unroll
        for (int i = 0; i < kRunE; ++i) {
          if (ok[i]) {
            uint32_t loc = 0;
            for (uint32_t j = 0; j < k; ++j)
              loc = loc * (byte_of(A.z, int(j)) + 1) + my[byte_of(A.y, int(j)) * QS + i * kBlock];
            const int32_t ti = tab + int32_t(loc);
            const uint32_t nw = nd[ti];
            for (uint32_t j = 0; j < k; ++j) my[byte_of(A.y, int(j)) * QS + i * kBlock] = uint8_t(nw >> (8 * j));
            if (!UNIT && !un[ti]) {
              a[i] = cmul(ph[ti], a[i]);
              changed[i] = true;
            }
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kRunE; ++i) {
      if (!active[i]) continue;
      uint64_t x = 0;
      for (int q = 0; q < nq; ++q) x += uint64_t(my[q * QS + i * kBlock]) * uint64_t(rq[q].stride);
      if (x != x0[i]) __builtin_nontemporal_store(int64_t(x), idx + e[i]);
      if (!UNIT && changed[i]) amp[e[i]] = a[i];
    }
  }
  if ((threadIdx.x & 63) == 0 && hits)
    atomicAdd(reinterpret_cast<unsigned long long*>(upd + (blockIdx.x & (kUpdSlots - 1))), (unsigned long long)hits);
}

// ------------------------------------------------------------------------------------------ dense gates
__global__ __launch_bounds__(kBlock) void k_table_clear(uint64_t* __restrict__ keys, int32_t* __restrict__ first, uint64_t H) {
  const uint64_t h = uint64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (h < H) {
    keys[h] = kEmpty;
    first[h] = INT32_MAX;
  }
}

__device__ __forceinline__ uint64_t hash_key(uint64_t key, uint32_t bits) {
  return (key * 0x9E3779B97F4A7C15ull) >> (64 - bits);   // Fibonacci hashing
}

// each matching entry finds (or claims) its slice key's slot; the slot keeps the smallest position
__global__ __launch_bounds__(kBlock) void k_insert(const int64_t* __restrict__ cnt, const int64_t* __restrict__ idx,
                                                   const Desc* __restrict__ g, const int64_t* __restrict__ off,
                                                   uint64_t* __restrict__ keys, int32_t* __restrict__ first,
                                                   uint32_t bits, int32_t* __restrict__ slot_of,
                                                   int32_t* __restrict__ loc_of, int64_t* __restrict__ misc) {
  const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= *cnt) return;
  const uint64_t x = uint64_t(idx[e]);
  uint32_t loc;
  if (!analyse(x, g, loc)) {
    slot_of[e] = -1;
    return;
  }
  const uint64_t key = x - uint64_t(off[loc]);
  const uint64_t mask = (uint64_t(1) << bits) - 1;
  uint64_t h = hash_key(key, bits);
  // at most half the slots are taken, so a free or equal slot turns up; the bound keeps the loop finite
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const uint64_t old = atomicCAS(reinterpret_cast<unsigned long long*>(keys + h), kEmpty, key);
    if (old == kEmpty || old == key) {
      slot_of[e] = int32_t(h);
      loc_of[e] = int32_t(loc);
      atomicMin(first + h, int32_t(e));
      return;
    }
    h = (h + 1) & mask;
  }
  slot_of[e] = -1;
  atomicOr(reinterpret_cast<unsigned long long*>(misc + kErr), 1ull);
}

// per-position counts of the two scans
struct LeaderCount {
  const int32_t* slot_of;
  const int32_t* first;
  __device__ int operator()(int64_t e) const {
    const int32_t s = slot_of[e];
    return s >= 0 && first[s] == int32_t(e) ? 1 : 0;
  }
};

struct OutCount {
  const int32_t* slot_of;
  const int32_t* first;
  const int32_t* sid;
  const double2* y;
  uint32_t dT;
  __device__ int operator()(int64_t e) const {
    const int32_t s = slot_of[e];
    if (s < 0) return 1;
    if (first[s] != int32_t(e)) return 0;
    const double2* ys = y + size_t(sid[s]) * dT;
    int c = 0;
    for (uint32_t i = 0; i < dT; ++i) c += nonzero(ys[i]) ? 1 : 0;
    return c;
  }
};

// pass 1 of a reduce-then-scan: the count of each chunk of kChunk positions
template <class F>
__global__ __launch_bounds__(kBlock) void k_chunk_sum(const int64_t* __restrict__ cnt, F f, int64_t* __restrict__ bsum) {
  __shared__ int sh[kBlock / 64];
  const int64_t n = *cnt, base = int64_t(blockIdx.x) * kChunk;
  int c = 0;
  for (int r = 0; r < kRounds; ++r) {
    const int64_t e = base + int64_t(r) * kBlock + threadIdx.x;
    if (e < n) c += f(e);
  }
  int total;
  (void)block_excl(c, sh, &total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// pass 2: exclusive scan of the nb chunk sums in place (one workgroup); the total goes to *tot
__global__ __launch_bounds__(kBlock) void k_top_scan(int64_t* __restrict__ bsum, int64_t nb, int64_t* __restrict__ tot) {
  __shared__ int64_t sh[kBlock / 64];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kBlock) {
    const int64_t b = b0 + threadIdx.x;
    const int64_t v = b < nb ? bsum[b] : 0;
    int64_t incl = v;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
    const int w = threadIdx.x >> 6;
    if (lane == 63) sh[w] = incl;
    __syncthreads();
    int64_t off = carry;
    for (int i = 0; i < w; ++i) off += sh[i];
    if (b < nb) bsum[b] = off + incl - v;
    carry += sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
  }
  if (threadIdx.x == 0) *tot = carry;
}

// pass 3 for the slice ranks: the leader (first entry) of each slice writes its rank
__global__ __launch_bounds__(kBlock) void k_rank_slices(const int64_t* __restrict__ cnt, LeaderCount f,
                                                        const int64_t* __restrict__ bsum, int32_t* __restrict__ sid) {
  __shared__ int sh[kBlock / 64];
  const int64_t n = *cnt, base = int64_t(blockIdx.x) * kChunk;
  int64_t pos = bsum[blockIdx.x];
  for (int r = 0; r < kRounds; ++r) {
    const int64_t e = base + int64_t(r) * kBlock + threadIdx.x;
    const int c = e < n ? f(e) : 0;
    int total;
    const int ex = block_excl(c, sh, &total);
    if (c) sid[f.slot_of[e]] = int32_t(pos + ex);
    pos += total;
  }
}

__global__ __launch_bounds__(kBlock) void k_zero2(double2* __restrict__ p, uint64_t count) {
  const uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < count) p[i] = make_double2(0.0, 0.0);
}

__global__ __launch_bounds__(kBlock) void k_gather(const int64_t* __restrict__ cnt, const double2* __restrict__ amp,
                                                   const int32_t* __restrict__ slot_of, const int32_t* __restrict__ loc_of,
                                                   const int32_t* __restrict__ sid, uint32_t dT, double2* __restrict__ x) {
  const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= *cnt) return;
  const int32_t s = slot_of[e];
  if (s >= 0) x[size_t(sid[s]) * dT + uint32_t(loc_of[e])] = amp[e];
}

// y[s, i] = sum_j U[i, j] x[s, j], j increasing from +0.0
__global__ __launch_bounds__(kBlock) void k_mix(const double2* __restrict__ x, const double2* __restrict__ U,
                                                uint64_t count, uint32_t dT, double2* __restrict__ y) {
#pragma clang fp contract(off)
  const uint64_t t = uint64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= count) return;
  const uint64_t s = t / dT;
  const uint32_t i = uint32_t(t - s * dT);
  const double2* xs = x + s * dT;
  const double2* ui = U + size_t(i) * dT;
  double re = 0.0, im = 0.0;
  for (uint32_t j = 0; j < dT; ++j) {
    const double2 p = cmul(ui[j], xs[j]);
    re = re + p.x;
    im = im + p.y;
  }
  y[t] = make_double2(re, im);
}

// pass 3 for the outputs: non-matching entries copy themselves, a slice's leader writes the slice's
// non-zero outputs by increasing row
__global__ __launch_bounds__(kBlock) void k_emit(const int64_t* __restrict__ cnt, OutCount f, const int64_t* __restrict__ bsum,
                                                 const int64_t* __restrict__ idx, const double2* __restrict__ amp,
                                                 const int32_t* __restrict__ loc_of, const int64_t* __restrict__ off,
                                                 int64_t* __restrict__ oidx, double2* __restrict__ oamp,
                                                 int64_t* __restrict__ upd) {
  __shared__ int sh[kBlock / 64];
  const int64_t n = *cnt, base = int64_t(blockIdx.x) * kChunk;
  int64_t pos = bsum[blockIdx.x];
  for (int r = 0; r < kRounds; ++r) {
    const int64_t e = base + int64_t(r) * kBlock + threadIdx.x;
    const int c = e < n ? f(e) : 0;
    int total;
    const int64_t p = pos + block_excl(c, sh, &total);
    wave_count(c && f.slot_of[e] >= 0 ? c : 0, upd);
    if (c) {
      const int32_t s = f.slot_of[e];
      if (s < 0) {
        oidx[p] = idx[e];
        oamp[p] = amp[e];
      } else {
        const int64_t key = idx[e] - off[loc_of[e]];
        const double2* ys = f.y + size_t(f.sid[s]) * f.dT;
        int64_t q = p;
        for (uint32_t i = 0; i < f.dT; ++i) {
          const double2 v = ys[i];
          if (nonzero(v)) {
            oidx[q] = key + off[i];
            oamp[q] = v;
            ++q;
          }
        }
      }
    }
    pos += total;
  }
}

// ------------------------------------------------------------------------------------------ readout
__global__ __launch_bounds__(kBlock) void k_norm_part(const int64_t* __restrict__ cnt, const double2* __restrict__ amp,
                                                      double* __restrict__ part) {
#pragma clang fp contract(off)
  __shared__ double sh[kBlock];
  const int64_t n = *cnt;
  double acc = 0.0;
  for (int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x; e < n; e += int64_t(gridDim.x) * kBlock) {
    const double2 a = amp[e];
    acc = acc + (a.x * a.x + a.y * a.y);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kBlock) void k_probs(const int64_t* __restrict__ cnt, const double2* __restrict__ amp,
                                                  double* __restrict__ p) {
#pragma clang fp contract(off)
  const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= *cnt) return;
  const double2 a = amp[e];
  p[e] = a.x * a.x + a.y * a.y;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_scatter_dense(const int64_t* __restrict__ cnt, const int64_t* __restrict__ idx,
                                                          const double2* __restrict__ amp, R* __restrict__ psi) {
  const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= *cnt) return;
  const double2 a = amp[e];
  const int64_t x = idx[e];
  psi[2 * x] = R(a.x);
  psi[2 * x + 1] = R(a.y);
}

// ------------------------------------------------------------------------------------------ host helpers
static unsigned blocks_for(int64_t n) { return unsigned(std::max<int64_t>(1, (n + kBlock - 1) / kBlock)); }

// grow a device buffer to `need` elements of T; the old one may still be read by queued work, so
// the stream drains before it is freed
template <typename T>
static int ensure(qd_sparse* s, DevBuf& b, size_t need) {
  if (b.p && b.cap >= need) return QD_OK;
  const size_t c = std::max<size_t>(need, b.cap ? b.cap * 2 : size_t(1) << 16);
  if (b.p) {
    QD_HIP(hipStreamSynchronize(s->stream));
    QD_HIP(hipFree(b.p));
    b.p = nullptr;
    b.cap = 0;
  }
  hipError_t e = hipMalloc(&b.p, c * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(QD_ENOMEM, "sparse workspace allocation failed (" + std::to_string(c * sizeof(T)) + " bytes)");
  }
  b.cap = c;
  return QD_OK;
}

template <typename T>
static T* P(const DevBuf& b) {
  return static_cast<T*>(b.p);
}

static int alloc_lists(qd_sparse* s, int64_t cap) {
  for (int b = 0; b < 2; ++b) {
    hipError_t e1 = hipMalloc((void**)&s->idx[b], size_t(cap) * sizeof(int64_t));
    hipError_t e2 = e1 == hipSuccess ? hipMalloc((void**)&s->amp[b], size_t(cap) * sizeof(double2)) : e1;
    if (e2 != hipSuccess) {
      (void)hipGetLastError();
      return fail(QD_ENOMEM, "sparse list allocation failed (" + std::to_string(cap) + " entries)");
    }
  }
  s->cap = cap;
  return QD_OK;
}

static void free_lists(qd_sparse* s) {
  for (int b = 0; b < 2; ++b) {
    if (s->idx[b]) (void)hipFree(s->idx[b]);
    if (s->amp[b]) (void)hipFree(s->amp[b]);
    s->idx[b] = nullptr;
    s->amp[b] = nullptr;
  }
  s->cap = 0;
}

// both list buffers hold at least `need` entries; the live list (count n) moves over
static int grow_lists(qd_sparse* s, int64_t need, int64_t n) {
  if (need <= s->cap) return QD_OK;
  if (need > kMaxEntries) return fail(QD_EOVERFLOW, "sparse state would exceed 2^31 - 1 entries");
  const int64_t cap = std::min<int64_t>(kMaxEntries, std::max<int64_t>(need, 2 * s->cap));
  int64_t* oi = s->idx[s->cur];
  double2* oa = s->amp[s->cur];
  int64_t* other_i = s->idx[1 - s->cur];
  double2* other_a = s->amp[1 - s->cur];
  int64_t* ni[2] = {nullptr, nullptr};
  double2* na[2] = {nullptr, nullptr};
  for (int b = 0; b < 2; ++b) {
    hipError_t e1 = hipMalloc((void**)&ni[b], size_t(cap) * sizeof(int64_t));
    hipError_t e2 = e1 == hipSuccess ? hipMalloc((void**)&na[b], size_t(cap) * sizeof(double2)) : e1;
    if (e2 != hipSuccess) {
      (void)hipGetLastError();
      for (int q = 0; q < 2; ++q) {
        if (ni[q]) (void)hipFree(ni[q]);
        if (na[q]) (void)hipFree(na[q]);
      }
      return fail(QD_ENOMEM, "sparse list allocation failed (" + std::to_string(cap) + " entries)");
    }
  }
  if (n > 0) {
    QD_HIP(hipMemcpyAsync(ni[s->cur], oi, size_t(n) * sizeof(int64_t), hipMemcpyDeviceToDevice, s->stream));
    QD_HIP(hipMemcpyAsync(na[s->cur], oa, size_t(n) * sizeof(double2), hipMemcpyDeviceToDevice, s->stream));
  }
  QD_HIP(hipStreamSynchronize(s->stream));
  (void)hipFree(oi);
  (void)hipFree(oa);
  (void)hipFree(other_i);
  (void)hipFree(other_a);
  for (int b = 0; b < 2; ++b) {
    s->idx[b] = ni[b];
    s->amp[b] = na[b];
  }
  s->cap = cap;
  return QD_OK;
}

// copy the device words to the pinned mirror and wait
static int read_misc(qd_sparse* s) {
  QD_HIP(hipMemcpyAsync(s->hmisc, s->misc, kMisc * sizeof(int64_t), hipMemcpyDeviceToHost, s->stream));
  QD_HIP(hipStreamSynchronize(s->stream));
  return QD_OK;
}

static int exact_count(qd_sparse* s, int64_t* n) {
  int rc = read_misc(s);
  if (rc) return rc;
  *n = s->hmisc[kCnt0 + s->cur];
  s->bound = *n;
  return QD_OK;
}

static Desc make_desc(const Register& r, const GatePlan& p) {
  Desc g{};
  g.k = uint32_t(p.k);
  g.m = uint32_t(p.m);
  g.dT = uint32_t(p.dT);
  auto fill = [&](Qudit& q, int w, int v) {
    q.ms = make_magic64(uint64_t(r.strides[w]));
    q.md = make_magic64(uint64_t(r.dims[w]));
    q.d = uint32_t(r.dims[w]);
    q.v = v;
  };
  for (int j = 0; j < p.k; ++j) fill(g.q[j], p.targets[j], 0);
  for (int j = 0; j < p.m; ++j) fill(g.q[p.k + j], p.controls[j], p.cvals[j]);
  return g;
}

// flat offset of each local index (first target most significant)
static std::vector<int64_t> local_offsets(const Register& r, const GatePlan& p) {
  std::vector<int64_t> off(static_cast<size_t>(p.dT), 0);
  for (int loc = 0; loc < p.dT; ++loc) {
    int rest = loc;
    int64_t o = 0;
    for (int j = p.k - 1; j >= 0; --j) {
      const int d = r.dims[p.targets[j]];
      o += int64_t(rest % d) * r.strides[p.targets[j]];
      rest /= d;
    }
    off[size_t(loc)] = o;
  }
  return off;
}

// pack pieces into one parameter block (256-byte aligned parts) and push it through the ring
struct Pack {
  std::vector<char> buf;
  size_t add(const void* src, size_t bytes) {
    const size_t at = (buf.size() + 255) / 256 * 256;
    buf.resize(at + bytes);
    if (bytes) std::memcpy(buf.data() + at, src, bytes);
    return at;
  }
};

// bytes of a descriptor that the kernels read: the header and the gate's k + m qudits
static size_t desc_bytes(const Desc& g) { return offsetof(Desc, q) + size_t(g.k + g.m) * sizeof(Qudit); }

struct MonoLaunch {
  size_t o_g, o_d, o_p, o_u;
  bool all_unit;
};

// append a monomial gate's descriptor and tables to the parameter block
static MonoLaunch pack_monomial(qd_sparse* s, const GatePlan& p, const Desc& g, Pack& pk) {
  const int dT = p.dT;
  const std::vector<int64_t> off = local_offsets(s->reg, p);
  std::vector<int64_t> delta(static_cast<size_t>(dT));
  std::vector<double2> ph(static_cast<size_t>(dT));
  std::vector<uint8_t> unit(static_cast<size_t>(dT));
  bool all_unit = true;
  for (int c = 0; c < dT; ++c) {
    const int r = p.cls == QD_CLASS_DIAGONAL ? c : p.dst[size_t(c)];
    delta[size_t(c)] = off[size_t(r)] - off[size_t(c)];
    ph[size_t(c)] = make_double2(p.ph[2 * size_t(c)], p.ph[2 * size_t(c) + 1]);
    unit[size_t(c)] = ph[size_t(c)].x == 1.0 && ph[size_t(c)].y == 0.0;
    all_unit = all_unit && unit[size_t(c)];
  }
  MonoLaunch L{};
  L.o_g = pk.add(&g, desc_bytes(g));
  L.o_d = pk.add(delta.data(), delta.size() * sizeof(int64_t));
  L.o_p = all_unit ? 0 : pk.add(ph.data(), ph.size() * sizeof(double2));
  L.o_u = all_unit ? 0 : pk.add(unit.data(), unit.size());
  L.all_unit = all_unit;
  return L;
}

static int launch_monomial(qd_sparse* s, const MonoLaunch& L, char* b) {
  const unsigned grid = unsigned(std::max<int64_t>(1, (s->bound + kMonoE * kBlock - 1) / (kMonoE * kBlock)));
  const int64_t* cnt = s->misc + kCnt0 + s->cur;
  const Desc* dg = reinterpret_cast<const Desc*>(b + L.o_g);
  const int64_t* dd = reinterpret_cast<const int64_t*>(b + L.o_d);
  if (L.all_unit)
    hipLaunchKernelGGL(k_monomial<true>, dim3(grid), dim3(kBlock), 0, s->stream, cnt, s->idx[s->cur], s->amp[s->cur], dg, dd,
                       nullptr, nullptr, s->misc + kUpd);
  else
    hipLaunchKernelGGL(k_monomial<false>, dim3(grid), dim3(kBlock), 0, s->stream, cnt, s->idx[s->cur], s->amp[s->cur], dg, dd,
                       reinterpret_cast<const double2*>(b + L.o_p), reinterpret_cast<const uint8_t*>(b + L.o_u),
                       s->misc + kUpd);
  QD_HIP(hipGetLastError());
  return QD_OK;
}

static int apply_dense(qd_sparse* s, const GatePlan& p, const Desc& g) {
  const uint32_t dT = uint32_t(p.dT);
  const std::vector<int64_t> off = local_offsets(s->reg, p);
  std::vector<double2> U(size_t(dT) * dT);
  for (size_t i = 0; i < U.size(); ++i) U[i] = make_double2(p.U[2 * i], p.U[2 * i + 1]);
  Pack pk;
  const size_t o_g = pk.add(&g, desc_bytes(g));
  const size_t o_o = pk.add(off.data(), off.size() * sizeof(int64_t));
  const size_t o_u = pk.add(U.data(), U.size() * sizeof(double2));
  void* dev = nullptr;
  int rc = ring_push_stream(&s->ring, s->stream, pk.buf.data(), pk.buf.size(), &dev);
  if (rc) return rc;
  char* b = static_cast<char*>(dev);
  const Desc* dg = reinterpret_cast<const Desc*>(b + o_g);
  const int64_t* doff = reinterpret_cast<const int64_t*>(b + o_o);
  const double2* dU = reinterpret_cast<const double2*>(b + o_u);

  const int64_t nb0 = s->bound;                    // upper bound on the count
  if (nb0 == 0) return QD_OK;
  // table of at least 2 nb0 slots (at most 2^31, so slots fit int32; the keys never fill it)
  uint32_t bits = 6;
  while (bits < 31 && (uint64_t(1) << bits) < uint64_t(2 * nb0)) ++bits;
  const uint64_t H = uint64_t(1) << bits;
  const int64_t nchunks = (nb0 + kChunk - 1) / kChunk;
  if ((rc = ensure<uint64_t>(s, s->keys, H)) || (rc = ensure<int32_t>(s, s->first, H)) ||
      (rc = ensure<int32_t>(s, s->sid, H)) || (rc = ensure<int32_t>(s, s->slot_of, size_t(nb0))) ||
      (rc = ensure<int32_t>(s, s->loc_of, size_t(nb0))) || (rc = ensure<int64_t>(s, s->bsum, size_t(nchunks))))
    return rc;
  uint64_t* keys = P<uint64_t>(s->keys);
  int32_t* first = P<int32_t>(s->first);
  int32_t* sid = P<int32_t>(s->sid);
  int32_t* slot_of = P<int32_t>(s->slot_of);
  int32_t* loc_of = P<int32_t>(s->loc_of);
  int64_t* bsum = P<int64_t>(s->bsum);

  const int64_t* cnt = s->misc + kCnt0 + s->cur;
  int64_t* idx = s->idx[s->cur];
  double2* amp = s->amp[s->cur];
  hipLaunchKernelGGL(k_table_clear, dim3(blocks_for(int64_t(H))), dim3(kBlock), 0, s->stream, keys, first, H);
  hipLaunchKernelGGL(k_insert, dim3(blocks_for(nb0)), dim3(kBlock), 0, s->stream, cnt, idx, dg, doff, keys, first, bits,
                     slot_of, loc_of, s->misc);
  const LeaderCount lc{slot_of, first};
  hipLaunchKernelGGL(k_chunk_sum<LeaderCount>, dim3(unsigned(nchunks)), dim3(kBlock), 0, s->stream, cnt, lc, bsum);
  hipLaunchKernelGGL(k_top_scan, dim3(1), dim3(kBlock), 0, s->stream, bsum, nchunks, s->misc + kNs);
  hipLaunchKernelGGL(k_rank_slices, dim3(unsigned(nchunks)), dim3(kBlock), 0, s->stream, cnt, lc, bsum, sid);
  QD_HIP(hipGetLastError());
  if ((rc = read_misc(s))) return rc;
  const int64_t n = s->hmisc[kCnt0 + s->cur];
  const int64_t ns = s->hmisc[kNs];
  if (s->hmisc[kErr]) return fail(QD_EDEVICE, "sparse key table overflow");
  s->bound = n;
  if (ns == 0) return QD_OK;                       // no entry matches: the list is unchanged

  const int64_t out_bound = n + ns * (int64_t(dT) - 1);
  if ((rc = grow_lists(s, out_bound, n))) return rc;
  idx = s->idx[s->cur];
  amp = s->amp[s->cur];
  const uint64_t nx = uint64_t(ns) * dT;
  if ((rc = ensure<double2>(s, s->xbuf, nx)) || (rc = ensure<double2>(s, s->ybuf, nx))) return rc;
  double2* xb = P<double2>(s->xbuf);
  double2* yb = P<double2>(s->ybuf);
  hipLaunchKernelGGL(k_zero2, dim3(blocks_for(int64_t(nx))), dim3(kBlock), 0, s->stream, xb, nx);
  hipLaunchKernelGGL(k_gather, dim3(blocks_for(n)), dim3(kBlock), 0, s->stream, cnt, amp, slot_of, loc_of, sid, dT, xb);
  hipLaunchKernelGGL(k_mix, dim3(blocks_for(int64_t(nx))), dim3(kBlock), 0, s->stream, xb, dU, nx, dT, yb);
  const int64_t nch = (n + kChunk - 1) / kChunk;
  const OutCount oc{slot_of, first, sid, yb, dT};
  hipLaunchKernelGGL(k_chunk_sum<OutCount>, dim3(unsigned(nch)), dim3(kBlock), 0, s->stream, cnt, oc, bsum);
  hipLaunchKernelGGL(k_top_scan, dim3(1), dim3(kBlock), 0, s->stream, bsum, nch, s->misc + kCnt0 + (1 - s->cur));
  hipLaunchKernelGGL(k_emit, dim3(unsigned(nch)), dim3(kBlock), 0, s->stream, cnt, oc, bsum, idx, amp, loc_of, doff,
                     s->idx[1 - s->cur], s->amp[1 - s->cur], s->misc + kUpd);
  QD_HIP(hipGetLastError());
  s->cur = 1 - s->cur;
  s->bound = out_bound;
  return QD_OK;
}

static bool run_eligible(const GatePlan& p) {
  return p.k <= kRunK && p.m <= kRunM && 64 + 32 + size_t(p.dT) * 21 <= size_t(kRunStage);
}

// shift a > 0 when the gate is X_{+a} on one target with unit entries, else 0
static int shift_of(const GatePlan& p, const Register& r) {
  if (p.k != 1 || p.cls != QD_CLASS_MONOMIAL) return 0;
  const int d = r.dims[p.targets[0]];
  const int a = p.dst[0];
  if (a == 0) return 0;
  for (int c = 0; c < d; ++c)
    if (p.dst[size_t(c)] != (c + a) % d || p.ph[2 * size_t(c)] != 1.0 || p.ph[2 * size_t(c) + 1] != 0.0) return 0;
  return a;
}

struct RunLaunch {
  size_t o_stage, o_q;               // staged block and register table in the parameter block
  int32_t stage16, ng, o_nd, o_ph, o_un;
  bool all_unit;
};

// bytes a gate adds to a launch's staged block: its descriptor, and for a table gate d_T rows of
// packed digits (4 B), phases (16 B) and unit flags (1 B)
static size_t run_cost(const GatePlan& p, bool shift) { return 32 + (shift ? 0 : size_t(p.dT) * 21); }

// append fused-run launches for plans[b..e) to the parameter block, each staging at most kRunStage bytes
static void pack_runs(qd_sparse* s, const std::vector<GatePlan>& plans, size_t b, size_t e, Pack& pk,
                      std::vector<RunLaunch>& out) {
  const Register& r = s->reg;
  std::vector<RunQudit> Q(size_t(r.n));
  for (int q = 0; q < r.n; ++q) {
    Q[size_t(q)] = RunQudit{};
    Q[size_t(q)].md = make_magic64(uint64_t(r.dims[q]));
    Q[size_t(q)].stride = r.strides[q];
    Q[size_t(q)].d = uint32_t(r.dims[q]);
  }
  const size_t o_q = pk.add(Q.data(), Q.size() * sizeof(RunQudit));
  size_t i = b;
  while (i < e) {
    std::vector<RunGateC> G;
    std::vector<uint32_t> nd;
    std::vector<double2> ph;
    std::vector<uint8_t> un;
    size_t bytes = 64;                 // room for the alignment of three table parts
    bool all_unit = true;
    while (i < e) {
      const GatePlan& p = plans[i];
      const int sh = shift_of(p, r);
      const size_t c = run_cost(p, sh > 0);
      if (!G.empty() && bytes + c > size_t(kRunStage)) break;
      bytes += c;
      RunGateC g{};
      g.shift = uint8_t(sh);
      g.k = uint8_t(p.k);
      g.m = uint8_t(p.m);
      for (int j = 0; j < p.k; ++j) {
        g.tq[j] = uint8_t(p.targets[j]);
        g.td1[j] = uint8_t(r.dims[p.targets[j]] - 1);
      }
      for (int j = 0; j < p.m; ++j) {
        g.cq[j] = uint8_t(p.controls[j]);
        g.cv[j] = uint8_t(p.cvals[j]);
      }
      if (sh == 0) {
        g.tab = int32_t(nd.size());
        for (int col = 0; col < p.dT; ++col) {
          int row = p.cls == QD_CLASS_DIAGONAL ? col : p.dst[size_t(col)];
          uint32_t packed = 0;
          for (int j = p.k - 1; j >= 0; --j) {
            const int d = r.dims[p.targets[j]];
            packed |= uint32_t(row % d) << (8 * j);
            row /= d;
          }
          nd.push_back(packed);
          const double2 v = make_double2(p.ph[2 * size_t(col)], p.ph[2 * size_t(col) + 1]);
          ph.push_back(v);
          const bool u = v.x == 1.0 && v.y == 0.0;
          un.push_back(uint8_t(u));
          all_unit = all_unit && u;
        }
      }
      G.push_back(g);
      ++i;
    }
    // staged block: descriptors, packed digits, phases, unit flags (16-byte aligned parts)
    std::vector<char> blk;
    auto put = [&](const void* src, size_t n) {
      const size_t at = (blk.size() + 15) / 16 * 16;
      blk.resize(at + n);
      if (n) std::memcpy(blk.data() + at, src, n);
      return at;
    };
    RunLaunch L{};
    put(G.data(), G.size() * sizeof(RunGateC));
    L.o_nd = int32_t(put(nd.data(), nd.size() * sizeof(uint32_t)));
    L.o_ph = int32_t(put(ph.data(), ph.size() * sizeof(double2)));
    L.o_un = int32_t(put(un.data(), un.size()));
    blk.resize((blk.size() + 15) / 16 * 16);
    L.stage16 = int32_t(blk.size() / 16);
    L.o_stage = pk.add(blk.data(), blk.size());
    L.o_q = o_q;
    L.ng = int32_t(G.size());
    L.all_unit = all_unit;
    out.push_back(L);
  }
}

// E entries per thread (two measured fastest on gfx950: four cost occupancy, one leaves the
// per-gate descriptor work unshared); LDS = staged block + n x E x 256 digit bytes
template <int E>
static void launch_run_e(qd_sparse* s, const RunLaunch& L, char* b, int cus) {
  const int64_t need = (s->bound + E * kBlock - 1) / (E * kBlock);
  const unsigned grid = unsigned(std::max<int64_t>(1, std::min<int64_t>(need, int64_t(cus) * kRunBlocksPerCU)));
  const size_t lds = size_t(L.stage16) * 16 + size_t(s->reg.n) * E * kBlock;
  const int64_t* cnt = s->misc + kCnt0 + s->cur;
  auto* st = reinterpret_cast<const uint4*>(b + L.o_stage);
  auto* Qd = reinterpret_cast<const RunQudit*>(b + L.o_q);
  if (L.all_unit)
    hipLaunchKernelGGL((k_mono_run<true, E>), dim3(grid), dim3(kBlock), lds, s->stream, cnt, s->idx[s->cur], s->amp[s->cur],
                       st, L.stage16, L.ng, L.o_nd, L.o_ph, L.o_un, Qd, int32_t(s->reg.n), s->misc + kUpd);
  else
    hipLaunchKernelGGL((k_mono_run<false, E>), dim3(grid), dim3(kBlock), lds, s->stream, cnt, s->idx[s->cur], s->amp[s->cur],
                       st, L.stage16, L.ng, L.o_nd, L.o_ph, L.o_un, Qd, int32_t(s->reg.n), s->misc + kUpd);
}

static int launch_run(qd_sparse* s, const RunLaunch& L, char* b) {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  }
  launch_run_e<2>(s, L, b, cus);
  QD_HIP(hipGetLastError());
  return QD_OK;
}

// Apply validated gates in order. A run of consecutive monomial gates shares one parameter upload;
// stretches of at least kRunMin gates that a fused run can hold go through k_mono_run (one launch
// per kRunStage bytes of descriptors and tables), the others gate by gate. Dense gates go one by one.
static int apply_sequence(qd_sparse* s, const SparseGate* gs, size_t count) {
  size_t i = 0;
  while (i < count) {
    std::vector<GatePlan> plans;
    while (i < count) {
      GatePlan p;
      const SparseGate& g = gs[i];
      make_plan(s->reg, g.t.data(), int32_t(g.t.size()), g.c.data(), g.v.data(), int32_t(g.c.size()), g.U.data(), &p);
      if (p.cls == QD_CLASS_DENSE) {
        if (plans.empty()) {
          int rc = apply_dense(s, p, make_desc(s->reg, p));
          if (rc) return rc;
          ++i;
          continue;
        }
        break;
      }
      plans.push_back(std::move(p));
      ++i;
    }
    if (plans.empty()) continue;
    Pack pk;
    std::vector<std::pair<int, size_t>> order;   // (0 = single gate, 1 = fused run), launch index
    std::vector<MonoLaunch> single;
    std::vector<RunLaunch> runs;
    size_t j = 0;
    while (j < plans.size()) {
      size_t e = j;
      while (e < plans.size() && run_eligible(plans[e])) ++e;
      if (e - j >= size_t(kRunMin)) {
        const size_t r0 = runs.size();
        pack_runs(s, plans, j, e, pk, runs);
        for (size_t q = r0; q < runs.size(); ++q) order.emplace_back(1, q);
        j = e;
      } else {
        single.push_back(pack_monomial(s, plans[j], make_desc(s->reg, plans[j]), pk));
        order.emplace_back(0, single.size() - 1);
        ++j;
      }
    }
    void* dev = nullptr;
    int rc = ring_push_stream(&s->ring, s->stream, pk.buf.data(), pk.buf.size(), &dev);
    if (rc) return rc;
    for (const auto& o : order) {
      rc = o.first ? launch_run(s, runs[o.second], static_cast<char*>(dev))
                   : launch_monomial(s, single[o.second], static_cast<char*>(dev));
      if (rc) return rc;
    }
  }
  return QD_OK;
}

}  // namespace sp

int sparse_apply_gates(qd_sparse* s, const SparseGate* gates, size_t count, uint32_t flags) {
  if (!s || (count && !gates)) return fail(QD_EINVAL, "null argument");
  for (size_t i = 0; i < count; ++i) {
    const SparseGate& g = gates[i];
    if (g.c.size() != g.v.size()) return fail(QD_EINVAL, "controls and control values differ in length");
    int rc = validate_gate(s->reg, g.t.data(), int32_t(g.t.size()), g.c.data(), g.v.data(), int32_t(g.c.size()),
                           g.U.data(), flags);
    if (rc) return rc;
  }
  (void)hipSetDevice(s->device);
  return sp::apply_sequence(s, gates, count);
}

}  // namespace qd

const qd::Register& qd::sparse_register(const qd_sparse* s) { return s->reg; }

using namespace qd;
using namespace qd::sp;

// ------------------------------------------------------------------------------------------ API
extern "C" {

void qd_sparse_free(qd_sparse* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  free_lists(s);
  if (s->misc) (void)hipFree(s->misc);
  if (s->hmisc) (void)hipHostFree(s->hmisc);
  for (DevBuf* b : {&s->keys, &s->first, &s->sid, &s->slot_of, &s->loc_of, &s->bsum, &s->xbuf, &s->ybuf})
    if (b->p) (void)hipFree(b->p);
  ring_free(&s->ring);
  delete s;
}

int qd_sparse_init(const int32_t* dims, int32_t n, int64_t capacity, void* hip_stream, qd_sparse** out) {
  if (!out) return fail(QD_EINVAL, "null output handle");
  if (capacity < 0 || capacity > kMaxEntries) return fail(QD_EINVAL, "capacity must be 0..2^31-1 entries");
  auto* s = new qd_sparse();
  int rc = make_register(dims, n, &s->reg);
  if (rc) {
    delete s;
    return rc;
  }
  s->stream = (hipStream_t)hip_stream;
  (void)hipGetDevice(&s->device);
  const int64_t cap = capacity ? capacity : int64_t(1) << 16;
  if ((rc = alloc_lists(s, cap)) != QD_OK) {
    qd_sparse_free(s);
    return rc;
  }
  if (hipMalloc((void**)&s->misc, kMisc * sizeof(int64_t)) != hipSuccess ||
      hipHostMalloc((void**)&s->hmisc, kMisc * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    qd_sparse_free(s);
    return fail(QD_ENOMEM, "sparse counter allocation failed");
  }
  std::memset(s->hmisc, 0, kMisc * sizeof(int64_t));
  s->hmisc[kCnt0] = 1;                              // |0...0>, amplitude 1
  const int64_t zero = 0;
  const double2 one = make_double2(1.0, 0.0);
  hipError_t e = hipMemcpyAsync(s->misc, s->hmisc, kMisc * sizeof(int64_t), hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(s->idx[0], &zero, sizeof(zero), hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(s->amp[0], &one, sizeof(one), hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) {
    qd_sparse_free(s);
    return hip_fail(e, "qd_sparse_init");
  }
  s->cur = 0;
  s->bound = 1;
  *out = s;
  return QD_OK;
}

int qd_sparse_upload(qd_sparse* s, const int64_t* idx, const double* amps, int64_t count) {
  if (!s || (count > 0 && (!idx || !amps))) return fail(QD_EINVAL, "null argument");
  if (count < 0 || count > kMaxEntries) return fail(QD_EINVAL, "entry count must be 0..2^31-1");
  std::vector<int64_t> sorted(idx, idx + count);
  for (int64_t e = 0; e < count; ++e) {
    if (idx[e] < 0 || idx[e] >= s->reg.D) return fail(QD_EINVAL, "index outside 0..D-1");
    const double re = amps[2 * e], im = amps[2 * e + 1];
    if (!std::isfinite(re) || !std::isfinite(im)) return fail(QD_EINVAL, "amplitude is not finite");
    if (re == 0.0 && im == 0.0) return fail(QD_EINVAL, "a stored amplitude must not be exactly zero");
  }
  std::sort(sorted.begin(), sorted.end());
  if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) return fail(QD_EINVAL, "duplicate index");
  QD_HIP(hipStreamSynchronize(s->stream));
  if (count > s->cap) {
    free_lists(s);
    int rc = alloc_lists(s, count);
    if (rc) return rc;
  }
  s->cur = 0;
  if (count > 0) {
    QD_HIP(hipMemcpy(s->idx[0], idx, size_t(count) * sizeof(int64_t), hipMemcpyHostToDevice));
    QD_HIP(hipMemcpy(s->amp[0], amps, size_t(count) * sizeof(double2), hipMemcpyHostToDevice));
  }
  s->hmisc[kCnt0] = count;
  QD_HIP(hipMemcpy(s->misc + kCnt0, s->hmisc + kCnt0, sizeof(int64_t), hipMemcpyHostToDevice));
  s->bound = count;
  return QD_OK;
}

int qd_sparse_set_basis(qd_sparse* s, const int32_t* values) {
  if (!s || !values) return fail(QD_EINVAL, "null argument");
  int64_t x = 0;
  for (int i = 0; i < s->reg.n; ++i) {
    if (values[i] < 0 || values[i] >= s->reg.dims[i]) return fail(QD_EINVAL, "basis value outside 0..d-1");
    x += int64_t(values[i]) * s->reg.strides[i];
  }
  const double one[2] = {1.0, 0.0};
  return qd_sparse_upload(s, &x, one, 1);
}

int qd_sparse_apply_gate(qd_sparse* s, const int32_t* targets, int32_t k, const int32_t* controls,
                         const int32_t* control_values, int32_t m, const double* U, uint32_t flags) {
  if (!s) return fail(QD_EINVAL, "null sparse state");
  // the copies below read the caller's arrays only after validation has checked them
  int rc = validate_gate(s->reg, targets, k, controls, control_values, m, U, flags);
  if (rc) return rc;
  SparseGate g;
  g.t.assign(targets, targets + k);
  if (m > 0) {
    g.c.assign(controls, controls + m);
    g.v.assign(control_values, control_values + m);
  }
  int64_t dT = 1;
  for (int j = 0; j < k; ++j) dT *= s->reg.dims[targets[j]];
  g.U.assign(U, U + 2 * size_t(dT) * size_t(dT));
  return sparse_apply_gates(s, &g, 1, flags);
}

int qd_sparse_apply_gates(qd_sparse* s, const qd_gate* gates, int32_t count, uint32_t flags) {
  if (!s || count < 0 || (count > 0 && !gates)) return fail(QD_EINVAL, "null argument or negative count");
  std::vector<SparseGate> seq(static_cast<size_t>(count));
  for (int32_t i = 0; i < count; ++i) {
    const qd_gate& g = gates[i];
    int rc = validate_gate(s->reg, g.targets, g.k, g.controls, g.control_values, g.m, g.U, flags);
    if (rc) return rc;
    SparseGate& q = seq[size_t(i)];
    q.t.assign(g.targets, g.targets + g.k);
    if (g.m > 0) {
      q.c.assign(g.controls, g.controls + g.m);
      q.v.assign(g.control_values, g.control_values + g.m);
    }
    int64_t dT = 1;
    for (int j = 0; j < g.k; ++j) dT *= s->reg.dims[g.targets[j]];
    q.U.assign(g.U, g.U + 2 * size_t(dT) * size_t(dT));
  }
  // every gate passed the checks above; the second pass only repeats the cheap ones
  return sparse_apply_gates(s, seq.data(), seq.size(), flags | QD_FLAG_SKIP_UNITARY_CHECK);
}

int qd_sparse_count(qd_sparse* s, int64_t* out) {
  if (!s || !out) return fail(QD_EINVAL, "null argument");
  return exact_count(s, out);
}

int qd_sparse_download(qd_sparse* s, int64_t* idx, double* amps, int64_t cap, int64_t* count) {
  if (!s || !count) return fail(QD_EINVAL, "null argument");
  int64_t n = 0;
  int rc = exact_count(s, &n);
  if (rc) return rc;
  *count = n;
  if (n > cap) return fail(QD_EINVAL, "output arrays hold fewer entries than the state");
  if (n > 0) {
    if (!idx || !amps) return fail(QD_EINVAL, "null output arrays");
    QD_HIP(hipMemcpy(idx, s->idx[s->cur], size_t(n) * sizeof(int64_t), hipMemcpyDeviceToHost));
    QD_HIP(hipMemcpy(amps, s->amp[s->cur], size_t(n) * sizeof(double2), hipMemcpyDeviceToHost));
  }
  return QD_OK;
}

int qd_sparse_device_lists(qd_sparse* s, int64_t** idx, double** amps, int64_t* count) {
  if (!s || !idx || !amps || !count) return fail(QD_EINVAL, "null argument");
  int rc = exact_count(s, count);
  if (rc) return rc;
  *idx = s->idx[s->cur];
  *amps = reinterpret_cast<double*>(s->amp[s->cur]);
  return QD_OK;
}

int qd_sparse_norm2(qd_sparse* s, double* out) {
  if (!s || !out) return fail(QD_EINVAL, "null argument");
  int64_t n = 0;
  int rc = exact_count(s, &n);
  if (rc) return rc;
  const unsigned grid = unsigned(std::max<int64_t>(1, std::min<int64_t>(1024, (n + kBlock * 8 - 1) / (kBlock * 8))));
  double* part = nullptr;
  QD_HIP(hipMalloc((void**)&part, grid * sizeof(double)));
  hipLaunchKernelGGL(k_norm_part, dim3(grid), dim3(kBlock), 0, s->stream, s->misc + kCnt0 + s->cur, s->amp[s->cur], part);
  std::vector<double> h(grid);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), part, grid * sizeof(double), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  (void)hipFree(part);
  if (e != hipSuccess) return hip_fail(e, "qd_sparse_norm2");
  double acc = 0.0;
  for (unsigned b = 0; b < grid; ++b) acc += h[b];    // fixed order over a grid fixed by the count
  *out = acc;
  return QD_OK;
}

int qd_sparse_probabilities(qd_sparse* s, double* out, int32_t out_is_device, int64_t cap) {
  if (!s || !out) return fail(QD_EINVAL, "null argument");
  int64_t n = 0;
  int rc = exact_count(s, &n);
  if (rc) return rc;
  if (n > cap) return fail(QD_EINVAL, "output array holds fewer entries than the state");
  if (n == 0) return QD_OK;
  double* dst = out;
  if (!out_is_device) QD_HIP(hipMalloc((void**)&dst, size_t(n) * sizeof(double)));
  hipLaunchKernelGGL(k_probs, dim3(blocks_for(n)), dim3(kBlock), 0, s->stream, s->misc + kCnt0 + s->cur, s->amp[s->cur], dst);
  hipError_t e = hipGetLastError();
  if (!out_is_device) {
    if (e == hipSuccess) e = hipMemcpyAsync(out, dst, size_t(n) * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(dst);
  } else if (e == hipSuccess) {
    e = hipStreamSynchronize(s->stream);
  }
  if (e != hipSuccess) return hip_fail(e, "qd_sparse_probabilities");
  return QD_OK;
}

int qd_sparse_to_dense(qd_sparse* s, qd_state* dst) {
  if (!s || !dst) return fail(QD_EINVAL, "null argument");
  if (dst->reg.n != s->reg.n || !std::equal(s->reg.dims, s->reg.dims + s->reg.n, dst->reg.dims))
    return fail(QD_EDIM, "dense state's register differs from the sparse state's");
  int64_t n = 0;
  int rc = exact_count(s, &n);
  if (rc) return rc;
  // the dense state's stream waits for nothing else: both calls run in order on the host
  if ((rc = launch_fill_basis(dst, -1))) return rc;
  QD_HIP(hipStreamSynchronize(dst->stream));
  if (n > 0) {
    if (dst->prec == QD_C128)
      hipLaunchKernelGGL(k_scatter_dense<double>, dim3(blocks_for(n)), dim3(kBlock), 0, s->stream, s->misc + kCnt0 + s->cur,
                         s->idx[s->cur], s->amp[s->cur], reinterpret_cast<double*>(dst->data));
    else
      hipLaunchKernelGGL(k_scatter_dense<float>, dim3(blocks_for(n)), dim3(kBlock), 0, s->stream, s->misc + kCnt0 + s->cur,
                         s->idx[s->cur], s->amp[s->cur], reinterpret_cast<float*>(dst->data));
    QD_HIP(hipGetLastError());
  }
  QD_HIP(hipStreamSynchronize(s->stream));
  return QD_OK;
}

int qd_sparse_updates(qd_sparse* s, int64_t* out) {
  if (!s || !out) return fail(QD_EINVAL, "null argument");
  int rc = read_misc(s);
  if (rc) return rc;
  int64_t t = 0;
  for (int i = 0; i < kUpdSlots; ++i) t += s->hmisc[kUpd + i];
  *out = t;
  return QD_OK;
}

int qd_sparse_sync(qd_sparse* s) {
  if (!s) return fail(QD_EINVAL, "null argument");
  QD_HIP(hipStreamSynchronize(s->stream));
  return QD_OK;
}

}  // extern "C"
