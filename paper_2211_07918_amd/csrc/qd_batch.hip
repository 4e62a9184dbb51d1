// Batched circuits: many independent registers of different sizes in one device arena, advanced
// one gate layer (the paper's Moment, Sec. 3.5) at a time by ONE launch per layer.
//
// A layer holds at most one single-target gate (optionally with one control) per circuit; a
// circuit's consecutive gates may also be composed on the host into one operation on up to four
// qudits (qd_batch_apply_layers). The host turns each circuit's operation into a descriptor
// (arena offset, slice map, slice offsets, U) and a prefix sum of work tiles (a tile is
// `block x spt` consecutive slices of one circuit), plus a table giving each tile's circuit. A
// workgroup copies its tile's descriptor and U to LDS and walks the tile, so heterogeneous
// registers and gates share one launch with divergence only between tiles, never inside a
// wavefront. Launches can be recorded into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "qd_internal.h"

namespace qd {

constexpr int kBatchMaxDim = 8;     // target dimension of a gate given to a layer
constexpr int kBatchMaxTargets = 4; // targets of a fused operation (its union of qudits)
constexpr int kBatchMaxSlice = 32;  // amplitudes per slice (d_T) of an operation
constexpr int kBatchGroups = kBatchMaxTargets + 1;
constexpr int kBatchMaxFuse = 8;    // gates composed into one operation

struct BatchDesc {
  int64_t off;                      // arena offset of the circuit's state (amplitudes)
  int64_t base;                     // control offset inside the state
  int64_t st;                       // target stride of a one-gate operation, 0 for a composed one
  uint32_t nwork;                   // active slices
  uint32_t tile0;                   // first global tile of this circuit
  int32_t dt;                       // slice size d_T, 0 = nothing for this circuit in this launch
  int32_t ng;                       // slice-map groups
  uint32_t uoff;                    // offset of U in the launch's value pool
  uint32_t spt;                     // slices per thread of a tile
  uint32_t gdim[kBatchGroups];
  uint32_t pad2[kBatchGroups & 1 ? 1 : 2];
  Magic32 gmag[kBatchGroups];
  int64_t gstride[kBatchGroups];
  int64_t yoff[kBatchMaxSlice];     // offset of local index y inside a slice
};

template <typename R>
struct BatchArgs {
  R* arena;
  const BatchDesc* desc;
  const R* upool;
  const uint32_t* tmap;             // circuit of each tile
  uint32_t ncirc;
  uint32_t ntiles;
};

template <typename R> struct CxB;
template <> struct CxB<double> { using T = double2; };
template <> struct CxB<float> { using T = float2; };

// NG: the most groups the descriptor can have (one target and one control leave at most 3 runs)
template <int NG>
__device__ __forceinline__ int64_t bd_offset(const BatchDesc& d, uint32_t idx) {
  int64_t off = d.base;
  uint32_t rem = idx;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    if (g < d.ng) {
      const uint32_t q = (g + 1 < d.ng) ? magic_div(rem, d.gmag[g]) : 0u;
      off += int64_t(rem - q * d.gdim[g]) * d.gstride[g];
      rem = q;
    }
  }
  return off;
}

// a thread takes the slices j0 + tid + k blockDim (k < spt <= 8) of the tile, in batches of
// at most 16 / DT slices whose loads are all issued before the first store (the register peak of
// the kernel stays that of about 16 amplitudes whatever the gate's dimension); spt is capped at two
// such batches, so a wide slice does not make a thread wait on several load round trips in turn
constexpr int kBatchMaxSpt = 8;
constexpr int batch_kb(int dt) { return (16 / dt) < 1 ? 1 : ((16 / dt) > kBatchMaxSpt ? kBatchMaxSpt : (16 / dt)); }

#ifndef QD_BATCH_LD
#define QD_BATCH_LD(p) (*(p))
#define QD_BATCH_ST(p, v) (*(p) = (v))
#endif

// FUSED: slice offsets from the descriptor's table; else y times the one target's stride
// d and U sit in LDS (copied per tile): global loads issued after the tile's first stores to the
// arena could not be served from the scalar cache and would be repeated as vector loads
template <typename R, int DT, bool FUSED>
__device__ __forceinline__ void batch_tile(const BatchArgs<R>& a, const BatchDesc& d, const R* U, uint32_t j0,
                                           uint32_t j1) {
  using C = typename CxB<R>::T;
  constexpr int KB = batch_kb(DT);
  C* psi = reinterpret_cast<C*>(a.arena) + d.off;
  const int spt = int(d.spt);
  for (int k0 = 0; k0 < spt; k0 += KB) {
    // the LDS values are re-read where used (held in registers they would take hundreds of them)
    __asm__ volatile("" ::: "memory");
    int64_t b[KB];
    C x[KB][DT];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const uint32_t j = j0 + threadIdx.x + uint32_t(k0 + k) * blockDim.x;
      b[k] = (k0 + k < spt && j < j1) ? bd_offset<FUSED ? kBatchGroups : 3>(d, j) : -1;
      if (b[k] >= 0) {
#pragma unroll
        for (int y = 0; y < DT; ++y) x[k][y] = QD_BATCH_LD(psi + (b[k] + (FUSED ? d.yoff[y] : y * d.st)));
      }
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      if (b[k] < 0) continue;
      auto row = [&](int r) {
        __asm__ volatile("" ::: "memory");
        R re = R(0), im = R(0);
#pragma unroll
        for (int c = 0; c < DT; ++c) {
          const R ur = U[2 * (r * DT + c)], ui = U[2 * (r * DT + c) + 1];
          re = fma(ur, x[k][c].x, re);
          re = fma(-ui, x[k][c].y, re);
          im = fma(ur, x[k][c].y, im);
          im = fma(ui, x[k][c].x, im);
        }
        C yv;
        yv.x = re;
        yv.y = im;
        QD_BATCH_ST(psi + (b[k] + (FUSED ? d.yoff[r] : r * d.st)), yv);
      };
      // composed slices of 6 or more amplitudes keep their rows as a loop: unrolled, the cases of
      // every slice size that share a launch would overflow the instruction cache
      if constexpr (FUSED && DT >= 6) {
#pragma unroll 1
        for (int r = 0; r < DT; ++r) row(r);
      } else {
#pragma unroll
        for (int r = 0; r < DT; ++r) row(r);
      }
    }
  }
}

// MAXDT = 0: a launch of one-gate operations only, addressed y times the target's stride; otherwise
// every operation of the launch (composed ones with slices of up to MAXDT = 16 or 32 amplitudes, and
// one-gate ones) is addressed through its offset table, so the variant holds one set of cases; the
// 32 variant (more registers) runs only launches that hold a slice above 16
template <int MAXDT> constexpr int batch_u_side() { return MAXDT > 16 ? kBatchMaxSlice : 16; }
template <typename R, int MAXDT>
__global__ __launch_bounds__(256) void k_batch_layer(BatchArgs<R> a) {
  const uint32_t per = (a.ntiles + gridDim.x - 1) / gridDim.x;
  const uint32_t t0 = blockIdx.x * per;
  const uint32_t t1 = min(a.ntiles, t0 + per);
  __shared__ BatchDesc d;
  __shared__ R sU[2 * batch_u_side<MAXDT>() * batch_u_side<MAXDT>()];
  static_assert(sizeof(BatchDesc) % 8 == 0, "descriptor copied in 8-byte words");
  for (uint32_t t = t0; t < t1; ++t) {
    const BatchDesc* gd = a.desc + a.tmap[t];
    __syncthreads();   // the previous tile is done with d and sU
    if (threadIdx.x < sizeof(BatchDesc) / 8)
      reinterpret_cast<uint64_t*>(&d)[threadIdx.x] = reinterpret_cast<const uint64_t*>(gd)[threadIdx.x];
    {
      const int nu = 2 * gd->dt * gd->dt;
      const R* gu = a.upool + gd->uoff;
      for (int i = int(threadIdx.x); i < nu; i += int(blockDim.x)) sU[i] = gu[i];
    }
    __syncthreads();
    const uint32_t tile_slices = blockDim.x * d.spt;
    const uint32_t j0 = (t - d.tile0) * tile_slices;
    const uint32_t j1 = min(d.nwork, j0 + tile_slices);
    if constexpr (MAXDT == 0) {
      switch (d.dt) {
        case 2: batch_tile<R, 2, false>(a, d, sU, j0, j1); break;
        case 3: batch_tile<R, 3, false>(a, d, sU, j0, j1); break;
        case 4: batch_tile<R, 4, false>(a, d, sU, j0, j1); break;
        case 5: batch_tile<R, 5, false>(a, d, sU, j0, j1); break;
        case 6: batch_tile<R, 6, false>(a, d, sU, j0, j1); break;
        case 7: batch_tile<R, 7, false>(a, d, sU, j0, j1); break;
        case 8: batch_tile<R, 8, false>(a, d, sU, j0, j1); break;
        default: break;
      }
    } else {
      switch (d.dt) {
        case 2: batch_tile<R, 2, true>(a, d, sU, j0, j1); break;
        case 3: batch_tile<R, 3, true>(a, d, sU, j0, j1); break;
        case 4: batch_tile<R, 4, true>(a, d, sU, j0, j1); break;
        case 5: batch_tile<R, 5, true>(a, d, sU, j0, j1); break;
        case 6: batch_tile<R, 6, true>(a, d, sU, j0, j1); break;
        case 7: batch_tile<R, 7, true>(a, d, sU, j0, j1); break;
        case 8: batch_tile<R, 8, true>(a, d, sU, j0, j1); break;
        case 9: batch_tile<R, 9, true>(a, d, sU, j0, j1); break;
        case 12: batch_tile<R, 12, true>(a, d, sU, j0, j1); break;
        case 16: batch_tile<R, 16, true>(a, d, sU, j0, j1); break;
        case 18: if constexpr (MAXDT >= 18) batch_tile<R, 18, true>(a, d, sU, j0, j1); break;
        case 24: if constexpr (MAXDT >= 24) batch_tile<R, 24, true>(a, d, sU, j0, j1); break;
        case 27: if constexpr (MAXDT >= 27) batch_tile<R, 27, true>(a, d, sU, j0, j1); break;
        case 32: if constexpr (MAXDT >= 32) batch_tile<R, 32, true>(a, d, sU, j0, j1); break;
        default: break;
      }
    }
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_batch_reset(R* arena, uint64_t total) {
  using C = typename CxB<R>::T;
  C* psi = reinterpret_cast<C*>(arena);
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += uint64_t(gridDim.x) * blockDim.x) {
    C v;
    v.x = R(0);
    v.y = R(0);
    psi[i] = v;
  }
}

// |0...0> of circuit c is the first amplitude of its state
template <typename R>
__global__ __launch_bounds__(256) void k_batch_ones(R* arena, const int64_t* offs, uint32_t ncirc) {
  using C = typename CxB<R>::T;
  C* psi = reinterpret_cast<C*>(arena);
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < ncirc; c += gridDim.x * blockDim.x) {
    C v;
    v.x = R(1);
    v.y = R(0);
    psi[offs[c]] = v;
  }
}

// ------------------------------------------------------------------------------------------ composition
// A circuit's consecutive gates composed into one operation on the union Q of their qudits (at most
// kBatchMaxTargets, d_Q <= kBatchMaxSlice): M = G_{w-1} ... G_0 in FP64 on the GPU, each G_i the gate
// embedded on Q (U where its control holds its value, the identity elsewhere), written to the
// launch's U pool in the state's precision. One workgroup per composed operation, M in LDS.
struct ComposeJob {
  uint32_t uoff;                    // offset of M in the launch's U pool (values of R)
  int32_t dq;                       // d_Q
  int32_t ng;                       // member gates, in circuit order
  uint32_t g0;                      // first member in the gate table
};
struct ComposeGate {
  int32_t tw;                       // weight of the target digit in Q's local index
  int32_t dt;                       // target dimension
  int32_t cw;                       // weight of the control digit, 0: no control
  int32_t cd;                       // control dimension
  int32_t cv;                       // control value
  uint32_t u64;                     // offset of U (dt x dt complex FP64, interleaved) in the FP64 pool
};

template <typename R>
__global__ __launch_bounds__(256) void k_batch_compose(const ComposeJob* __restrict__ jobs,
                                                       const ComposeGate* __restrict__ gates,
                                                       const double* __restrict__ u64, R* __restrict__ pool) {
  constexpr int kEnt = kBatchMaxSlice * kBatchMaxSlice / 256;   // entries of M per thread
  __shared__ double2 M[kBatchMaxSlice * kBatchMaxSlice];
  __shared__ double2 su[kBatchMaxDim * kBatchMaxDim];
  const ComposeJob J = jobs[blockIdx.x];
  const int dq = J.dq, n = dq * dq, tid = int(threadIdx.x);
  for (int e = tid; e < n; e += 256) M[e] = double2{(e / dq == e % dq) ? 1.0 : 0.0, 0.0};
  for (int gi = 0; gi < J.ng; ++gi) {
    const ComposeGate G = gates[J.g0 + gi];
    __syncthreads();   // M complete, su free
    for (int e = tid; e < G.dt * G.dt; e += 256) su[e] = double2{u64[G.u64 + 2 * e], u64[G.u64 + 2 * e + 1]};
    __syncthreads();
    double2 nv[kEnt];
#pragma unroll
    for (int q = 0; q < kEnt; ++q) {
      const int e = tid + 256 * q;
      if (e >= n) continue;
      const int x = e / dq, col = e - x * dq;
      const int yt = (x / G.tw) % G.dt;                       // target digit of row x
      nv[q] = M[e];
      if (G.cw == 0 || (x / G.cw) % G.cd == G.cv) {
        const int x0 = x - yt * G.tw;                         // row x with its target digit 0
        double re = 0.0, im = 0.0;
        for (int y = 0; y < G.dt; ++y) {
          const double2 u = su[yt * G.dt + y], m = M[(x0 + y * G.tw) * dq + col];
          re += u.x * m.x - u.y * m.y;
          im += u.x * m.y + u.y * m.x;
        }
        nv[q] = double2{re, im};
      }
    }
    __syncthreads();   // every row of M is read
#pragma unroll
    for (int q = 0; q < kEnt; ++q) {
      const int e = tid + 256 * q;
      if (e < n) M[e] = nv[q];
    }
  }
  __syncthreads();
  for (int e = tid; e < n; e += 256) {
    pool[J.uoff + 2 * e] = R(M[e].x);
    pool[J.uoff + 2 * e + 1] = R(M[e].y);
  }
}

}  // namespace qd

struct qd_batch {
  int prec = QD_C64;
  hipStream_t stream = nullptr;
  std::vector<qd::Register> regs;
  std::vector<int64_t> offs;
  int64_t total = 0;
  void* arena = nullptr;
  int64_t* offs_dev = nullptr;
  qd::ParamRing ring;
  // graph recording
  bool capturing = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t last = nullptr;
  std::vector<void*> layer_bufs;          // device buffers owned by recorded layers
  std::vector<std::vector<unsigned char>> layer_args;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> compose_ev;   // composition launches not yet timed
  double compose_ms = 0.0;                // time of earlier composition launches already read back
};

namespace qd {

template <typename R>
static void* batch_kernel_ptr(int maxdt) {
  if (maxdt == 0) return reinterpret_cast<void*>(k_batch_layer<R, 0>);
  return maxdt <= 16 ? reinterpret_cast<void*>(k_batch_layer<R, 16>) : reinterpret_cast<void*>(k_batch_layer<R, 32>);
}

static void free_graph(qd_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->last = nullptr;
  for (void* p : b->layer_bufs) (void)hipFree(p);
  b->layer_bufs.clear();
  b->layer_args.clear();
}

// exchange the recording state (graph, executable, owned layer buffers) of two batches
static void swap_graphs(qd_batch* a, qd_batch* b) {
  std::swap(a->capturing, b->capturing);
  std::swap(a->graph, b->graph);
  std::swap(a->exec, b->exec);
  std::swap(a->last, b->last);
  std::swap(a->layer_bufs, b->layer_bufs);
  std::swap(a->layer_args, b->layer_args);
}

static int batch_reset(qd_batch* b) {
  const unsigned grid = unsigned(std::min<uint64_t>((uint64_t(b->total) + 255) / 256, 65536));
  const uint32_t nc = uint32_t(b->regs.size());
  const unsigned g2 = std::max(1u, std::min(1024u, (nc + 255) / 256));
  if (b->prec == QD_C128) {
    hipLaunchKernelGGL((k_batch_reset<double>), dim3(grid), dim3(256), 0, b->stream, (double*)b->arena, uint64_t(b->total));
    hipLaunchKernelGGL((k_batch_ones<double>), dim3(g2), dim3(256), 0, b->stream, (double*)b->arena, b->offs_dev, nc);
  } else {
    hipLaunchKernelGGL((k_batch_reset<float>), dim3(grid), dim3(256), 0, b->stream, (float*)b->arena, uint64_t(b->total));
    hipLaunchKernelGGL((k_batch_ones<float>), dim3(g2), dim3(256), 0, b->stream, (float*)b->arena, b->offs_dev, nc);
  }
  QD_HIP(hipGetLastError());
  return QD_OK;
}

// One circuit's operation in a launch: up to kBatchMaxTargets targets (first most significant in
// U's local index), at most one control, U of d_T x d_T (FP64, interleaved). k = 0: nothing.
struct BatchOp {
  int k = 0;
  int32_t t[kBatchMaxTargets] = {};
  int m = 0;
  int32_t c = 0, v = 0;
  std::vector<double> U;                  // one gate: its U
  std::vector<const qd_gate*> members;    // composed (2 or more gates): composed on the GPU
};

static bool slice_supported(int dT) {
  return (dT >= 2 && dT <= 9) || dT == 12 || dT == 16 || dT == 18 || dT == 24 || dT == 27 || dT == 32;
}

// Host: descriptors and U pool of one launch; *ntiles the total tile count, *maxdt the largest slice
// of a composed operation (0 when the launch holds one-gate operations only).
struct ComposeWork {                    // the composed operations of one launch
  std::vector<ComposeJob> jobs;
  std::vector<ComposeGate> gates;
  std::vector<double> u64;
};

template <typename R>
static int build_layer(qd_batch* b, const std::vector<BatchOp>& ops, std::vector<BatchDesc>* desc,
                       std::vector<R>* pool, ComposeWork* cw, uint32_t* ntiles, int* maxdt) {
  *maxdt = 0;
  const uint32_t nc = uint32_t(b->regs.size());
  const TuneParams& tp = tune();
  desc->assign(nc, BatchDesc{});
  pool->clear();
  cw->jobs.clear();
  cw->gates.clear();
  cw->u64.clear();
  uint64_t tiles = 0;
  for (uint32_t c = 0; c < nc; ++c) {
    const Register& r = b->regs[c];
    BatchDesc& d = (*desc)[c];
    d.off = b->offs[c];
    d.tile0 = uint32_t(tiles);
    const BatchOp& o = ops[c];
    if (o.k == 0) continue;
    int role[QD_MAX_QUDITS] = {};
    int dT = 1;
    for (int j = 0; j < o.k; ++j) {
      role[o.t[j]] = 1;
      dT *= r.dims[o.t[j]];
    }
    if (!slice_supported(dT)) return fail(QD_EINVAL, "internal: unsupported batched slice size");
    int64_t base = 0;
    if (o.m == 1) {
      role[o.c] = 1;
      base = int64_t(o.v) * r.strides[o.c];
    }
    std::vector<Group> g = make_groups(r, role, nullptr, 0, r.n);
    if (int(g.size()) > kBatchGroups) return fail(QD_EINVAL, "internal: too many groups");
    uint64_t nwork = 1;
    for (size_t i = 0; i < g.size(); ++i) {
      d.gdim[i] = uint32_t(g[i].dim);
      d.gmag[i] = make_magic32(uint32_t(g[i].dim));
      d.gstride[i] = g[i].stride;
      nwork *= g[i].dim;
    }
    d.ng = int32_t(g.size());
    d.base = base;
    for (int y = 0; y < dT; ++y) {   // offset of local index y: its target digits times their strides
      int rest = y;
      int64_t off = 0;
      for (int j = o.k - 1; j >= 0; --j) {
        const int dj = r.dims[o.t[j]];
        off += int64_t(rest % dj) * r.strides[o.t[j]];
        rest /= dj;
      }
      d.yoff[y] = off;
    }
    d.dt = dT;
    d.st = o.k == 1 ? r.strides[o.t[0]] : 0;
    *maxdt = std::max(*maxdt, o.k == 1 ? 0 : dT);
    d.nwork = uint32_t(nwork);
    d.uoff = uint32_t(pool->size());
    if (o.members.empty()) {
      for (int i = 0; i < 2 * dT * dT; ++i) pool->push_back(R(o.U[size_t(i)]));
    } else {
      // composed on the GPU into this slot: the weights of Q's digits (first most significant)
      pool->resize(pool->size() + 2 * size_t(dT) * dT, R(0));
      int wt[QD_MAX_QUDITS] = {};
      {
        int w = 1;
        for (int j = o.k - 1; j >= 0; --j) {
          wt[o.t[j]] = w;
          w *= r.dims[o.t[j]];
        }
      }
      ComposeJob J;
      J.uoff = d.uoff;
      J.dq = dT;
      J.ng = int32_t(o.members.size());
      J.g0 = uint32_t(cw->gates.size());
      cw->jobs.push_back(J);
      for (const qd_gate* g : o.members) {
        ComposeGate G;
        const int t = g->targets[0];
        G.tw = wt[t];
        G.dt = r.dims[t];
        G.cw = g->m == 1 ? wt[g->controls[0]] : 0;
        G.cd = g->m == 1 ? r.dims[g->controls[0]] : 1;
        G.cv = g->m == 1 ? g->control_values[0] : 0;
        G.u64 = uint32_t(cw->u64.size());
        cw->u64.insert(cw->u64.end(), g->U, g->U + 2 * size_t(G.dt) * G.dt);
        cw->gates.push_back(G);
      }
    }
    // slices per thread: tuned per operation key, else per slice class, else the rule
    int64_t smin = INT64_MAX;
    for (int j = 0; j < o.k; ++j) smin = std::min<int64_t>(smin, r.strides[o.t[j]]);
    const int kv = tp.batch_spt_key[batch_key(!o.members.empty(), dT, smin)];
    const int cls = dT >= 12 ? tp.batch_spt_wide : (dT >= 5 ? tp.batch_spt_mid : 0);
    d.spt = uint32_t(kv ? kv : (cls ? cls : std::min(tp.batch_spt, 2 * batch_kb(dT))));
    const uint64_t tile_slices = uint64_t(tp.batch_block) * d.spt;
    tiles += (nwork + tile_slices - 1) / tile_slices;
    if (tiles > 0xFFFFFFF0ull) return fail(QD_EOVERFLOW, "too many tiles in one layer");
  }
  *ntiles = uint32_t(tiles);
  return QD_OK;
}

// A layer's gate for circuit c, validated (one target of dimension <= 8, at most one control).
static int layer_gate(const qd_batch* b, uint32_t c, const qd_gate& G) {
  if (G.k == 0) return QD_OK;
  if (G.k != 1 || G.m > 1) return fail(QD_EINVAL, "batched layers take one target and at most one control (circuit " + std::to_string(c) + ")");
  const Register& r = b->regs[c];
  int rc = validate_gate(r, G.targets, G.k, G.controls, G.control_values, G.m, G.U, 0);
  if (rc) return fail(rc, "circuit " + std::to_string(c) + ": " + qd_last_error());
  if (r.dims[G.targets[0]] > kBatchMaxDim) return fail(QD_EINVAL, "batched layers support target dimensions up to 8");
  return QD_OK;
}

static BatchOp op_of(const qd_batch* b, uint32_t c, const qd_gate& G) {
  BatchOp o;
  if (G.k == 0) return o;
  const int dt = b->regs[c].dims[G.targets[0]];
  o.k = 1;
  o.t[0] = G.targets[0];
  if (G.m == 1) {
    o.m = 1;
    o.c = G.controls[0];
    o.v = G.control_values[0];
  }
  o.U.assign(G.U, G.U + 2 * size_t(dt) * dt);
  return o;
}

// The union Q of the gates' qudits (targets and controls, ascending) and its dimension d_Q; false
// when it does not fit one slice.
static bool gate_union(const Register& r, const qd_gate* const* gs, int w, int* Q, int* nq_out, int* dQ_out) {
  int nq = 0;
  for (int i = 0; i < w; ++i) {
    Q[nq++] = gs[i]->targets[0];
    if (gs[i]->m == 1) Q[nq++] = gs[i]->controls[0];
  }
  std::sort(Q, Q + nq);
  nq = int(std::unique(Q, Q + nq) - Q);
  if (nq > kBatchMaxTargets) return false;
  int dQ = 1;
  for (int j = 0; j < nq; ++j) dQ *= r.dims[Q[j]];
  *nq_out = nq;
  *dQ_out = dQ;
  return slice_supported(dQ);
}

// The next block of circuit c's gates, from layer *cursor on (empty slots skipped): consecutive
// gates while the block has at most W of them and they compose on at most kBatchMaxTargets qudits
// with a supported slice size; a block of one gate stays that gate. *cursor moves past the block;
// out->k == 0 when the circuit has no gate left.
static void next_block(const qd_batch* b, uint32_t c, const qd_gate* gates, int32_t nlayers, int W,
                       int32_t* cursor, BatchOp* out) {
  const uint32_t nc = uint32_t(b->regs.size());
  const Register& r = b->regs[c];
  const qd_gate* cur[kBatchMaxFuse];
  int n = 0;
  int32_t l = *cursor;
  for (; l < nlayers; ++l) {
    const qd_gate& G = gates[size_t(l) * nc + c];
    if (G.k == 0) continue;
    if (n == 0) {
      cur[n++] = &G;
      continue;
    }
    if (n == W) break;
    cur[n] = &G;
    int Q[2 * kBatchMaxFuse], nq = 0, dQ = 0;
    if (!gate_union(r, cur, n + 1, Q, &nq, &dQ)) break;
    ++n;
  }
  *cursor = l;
  *out = BatchOp();
  if (n == 1) {
    *out = op_of(b, c, *cur[0]);
  } else if (n > 1) {   // fits one slice: checked as the block grew; composed on the GPU in FP64
    int Q[2 * kBatchMaxFuse], nq = 0, dQ = 0;
    (void)gate_union(r, cur, n, Q, &nq, &dQ);
    out->k = nq;
    for (int j = 0; j < nq; ++j) out->t[j] = Q[j];
    out->members.assign(cur, cur + n);
  }
}

template <typename R>
static int apply_layer_t(qd_batch* b, const std::vector<BatchOp>& ops) {
  std::vector<BatchDesc> desc;
  std::vector<R> pool;
  ComposeWork cw;
  uint32_t ntiles = 0;
  int maxdt = 0;
  int rc = build_layer<R>(b, ops, &desc, &pool, &cw, &ntiles, &maxdt);
  if (rc) return rc;
  auto pad256 = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t dbytes = desc.size() * sizeof(BatchDesc);
  const size_t pbytes = std::max<size_t>(pool.size(), 1) * sizeof(R);
  const size_t dpad = pad256(dbytes);
  const size_t ppad = pad256(pbytes);
  const size_t tpad = pad256(std::max<size_t>(ntiles, 1) * sizeof(uint32_t));
  const size_t jpad = pad256(cw.jobs.size() * sizeof(ComposeJob));
  const size_t gpad = pad256(cw.gates.size() * sizeof(ComposeGate));
  const size_t upad = pad256(cw.u64.size() * sizeof(double));
  std::vector<unsigned char> blob(dpad + ppad + tpad + jpad + gpad + upad, 0);
  std::memcpy(blob.data(), desc.data(), dbytes);
  if (!pool.empty()) std::memcpy(blob.data() + dpad, pool.data(), pool.size() * sizeof(R));
  uint32_t* tmap = reinterpret_cast<uint32_t*>(blob.data() + dpad + ppad);   // tile -> circuit
  unsigned char* cbase = blob.data() + dpad + ppad + tpad;
  if (!cw.jobs.empty()) {
    std::memcpy(cbase, cw.jobs.data(), cw.jobs.size() * sizeof(ComposeJob));
    std::memcpy(cbase + jpad, cw.gates.data(), cw.gates.size() * sizeof(ComposeGate));
    std::memcpy(cbase + jpad + gpad, cw.u64.data(), cw.u64.size() * sizeof(double));
  }
  // the composed operations of the launch, built in FP64 on the GPU into the launch's U pool
  // before the layer runs (timed with events, read back by qd_batch_compose_ms)
  auto compose = [&](unsigned char* dev) -> int {
    if (cw.jobs.empty()) return QD_OK;
    const size_t c0 = dpad + ppad + tpad;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (b->compose_ev.size() >= 1024) {   // fold older timings so the event list stays bounded
      for (auto& ev : b->compose_ev) {
        float t = 0.f;
        QD_HIP(hipEventSynchronize(ev.second));
        QD_HIP(hipEventElapsedTime(&t, ev.first, ev.second));
        b->compose_ms += t;
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
      }
      b->compose_ev.clear();
    }
    QD_HIP(hipEventCreate(&e0));
    QD_HIP(hipEventCreate(&e1));
    b->compose_ev.emplace_back(e0, e1);
    QD_HIP(hipEventRecord(e0, b->stream));
    hipLaunchKernelGGL((k_batch_compose<R>), dim3(unsigned(cw.jobs.size())), dim3(256), 0, b->stream,
                       reinterpret_cast<const ComposeJob*>(dev + c0),
                       reinterpret_cast<const ComposeGate*>(dev + c0 + jpad),
                       reinterpret_cast<const double*>(dev + c0 + jpad + gpad), reinterpret_cast<R*>(dev + dpad));
    QD_HIP(hipGetLastError());
    QD_HIP(hipEventRecord(e1, b->stream));
    return QD_OK;
  };
  for (uint32_t c = 0; c < uint32_t(desc.size()); ++c) {
    const uint32_t end = c + 1 < uint32_t(desc.size()) ? desc[c + 1].tile0 : ntiles;
    for (uint32_t t = desc[c].tile0; t < end; ++t) tmap[t] = c;
  }
  const TuneParams& tp = tune();
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  // batch_wpc persistent workgroups per compute unit walk the tile list; 64 = one workgroup per tile
  const int wpc = tune().batch_wpc;
  const unsigned grid = wpc >= 64 ? std::max(1u, ntiles)
                                  : std::max(1u, std::min<unsigned>(ntiles, unsigned(cus) * unsigned(wpc)));
  BatchArgs<R> a;
  a.arena = reinterpret_cast<R*>(b->arena);
  a.ncirc = uint32_t(desc.size());
  a.ntiles = ntiles;
  if (!b->capturing) {
    if (ntiles == 0) return QD_OK;
    void* dev_blob = nullptr;
    rc = ring_push_stream(&b->ring, b->stream, blob.data(), blob.size(), &dev_blob);
    if (rc) return rc;
    rc = compose(static_cast<unsigned char*>(dev_blob));
    if (rc) return rc;
    a.desc = reinterpret_cast<const BatchDesc*>(dev_blob);
    a.upool = reinterpret_cast<const R*>(static_cast<unsigned char*>(dev_blob) + dpad);
    a.tmap = reinterpret_cast<const uint32_t*>(static_cast<unsigned char*>(dev_blob) + dpad + ppad);
    if (maxdt == 0)
      hipLaunchKernelGGL((k_batch_layer<R, 0>), dim3(grid), dim3(tp.batch_block), 0, b->stream, a);
    else if (maxdt <= 16)
      hipLaunchKernelGGL((k_batch_layer<R, 16>), dim3(grid), dim3(tp.batch_block), 0, b->stream, a);
    else
      hipLaunchKernelGGL((k_batch_layer<R, 32>), dim3(grid), dim3(tp.batch_block), 0, b->stream, a);
    QD_HIP(hipGetLastError());
    return QD_OK;
  }
  // recording: the layer's parameters live in their own device buffer for the graph's lifetime
  void* buf = nullptr;
  QD_HIP(hipMalloc(&buf, blob.size()));
  b->layer_bufs.push_back(buf);
  QD_HIP(hipMemcpy(buf, blob.data(), blob.size(), hipMemcpyHostToDevice));
  rc = compose(static_cast<unsigned char*>(buf));   // once, at recording: replays reuse the blocks
  if (rc) return rc;
  if (ntiles == 0) return QD_OK;
  a.desc = reinterpret_cast<const BatchDesc*>(buf);
  a.upool = reinterpret_cast<const R*>(static_cast<unsigned char*>(buf) + dpad);
  a.tmap = reinterpret_cast<const uint32_t*>(static_cast<unsigned char*>(buf) + dpad + ppad);
  b->layer_args.emplace_back(sizeof(a));
  std::memcpy(b->layer_args.back().data(), &a, sizeof(a));
  void* kargs[1] = {b->layer_args.back().data()};
  hipKernelNodeParams kp{};
  kp.blockDim = dim3(tp.batch_block);
  kp.gridDim = dim3(grid);
  kp.func = batch_kernel_ptr<R>(maxdt);
  kp.kernelParams = kargs;
  kp.sharedMemBytes = 0;
  kp.extra = nullptr;
  hipGraphNode_t node;
  QD_HIP(hipGraphAddKernelNode(&node, b->graph, b->last ? &b->last : nullptr, b->last ? 1 : 0, &kp));
  b->last = node;
  return QD_OK;
}

}  // namespace qd

using namespace qd;

extern "C" {

int qd_batch_create(int32_t nc, const int32_t* n_per, const int32_t* dims_flat, int32_t prec, void* hip_stream,
                    qd_batch** out) {
  if (!out || !n_per || !dims_flat || nc < 1) return fail(QD_EINVAL, "bad batch arguments");
  if (prec != QD_C64 && prec != QD_C128) return fail(QD_EINVAL, "precision must be QD_C128 or QD_C64");
  auto* b = new qd_batch();
  b->prec = prec;
  b->stream = (hipStream_t)hip_stream;
  int64_t pos = 0, total = 0;
  for (int c = 0; c < nc; ++c) {
    Register r;
    int rc = make_register(dims_flat + pos, n_per[c], &r);
    if (rc) {
      delete b;
      return fail(rc, "circuit " + std::to_string(c) + ": " + qd_last_error());
    }
    if (r.D > int64_t(0xFFFFFFFFll)) {
      delete b;
      return fail(QD_EOVERFLOW, "batched registers must have D < 2^32");
    }
    pos += n_per[c];
    b->regs.push_back(r);
    b->offs.push_back(total);
    total += r.D;
  }
  b->total = total;
  const size_t bytes = size_t(total) * amp_bytes(prec);
  hipError_t e = hipMalloc(&b->arena, bytes);
  if (e == hipSuccess) e = hipMalloc((void**)&b->offs_dev, sizeof(int64_t) * nc);
  if (e == hipSuccess) e = hipMemcpy(b->offs_dev, b->offs.data(), sizeof(int64_t) * nc, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    qd_batch_free(b);
    return hip_fail(e, "batch arena");
  }
  int rc = batch_reset(b);
  if (rc) {
    qd_batch_free(b);
    return rc;
  }
  *out = b;
  return QD_OK;
}

int qd_batch_size(const qd_batch* b, int64_t* total) {
  if (!b || !total) return fail(QD_EINVAL, "null argument");
  *total = b->total;
  return QD_OK;
}

int qd_batch_offset(const qd_batch* b, int32_t c, int64_t* off) {
  if (!b || !off) return fail(QD_EINVAL, "null argument");
  if (c < 0 || c >= int32_t(b->offs.size())) return fail(QD_EINVAL, "circuit index out of range");
  *off = b->offs[c];
  return QD_OK;
}

int qd_batch_reset(qd_batch* b) {
  if (!b) return fail(QD_EINVAL, "null batch");
  return batch_reset(b);
}

int qd_batch_apply_layer(qd_batch* b, const qd_gate* gates) {
  if (!b || !gates) return fail(QD_EINVAL, "null argument");
  const uint32_t nc = uint32_t(b->regs.size());
  std::vector<BatchOp> ops(nc);
  for (uint32_t c = 0; c < nc; ++c) {
    int rc = layer_gate(b, c, gates[c]);
    if (rc) return rc;
    ops[c] = op_of(b, c, gates[c]);
  }
  return b->prec == QD_C128 ? apply_layer_t<double>(b, ops) : apply_layer_t<float>(b, ops);
}

int qd_batch_apply_layers(qd_batch* b, const qd_gate* gates, int32_t nlayers, int32_t width) {
  if (!b || (nlayers > 0 && !gates)) return fail(QD_EINVAL, "null argument");
  if (nlayers < 0 || width < 0 || width > kBatchMaxFuse) return fail(QD_EINVAL, "bad layer count or fusion width (0..8)");
  const int W = width ? width : tune().batch_fuse;
  const uint32_t nc = uint32_t(b->regs.size());
  for (int32_t l = 0; l < nlayers; ++l)
    for (uint32_t c = 0; c < nc; ++c) {
      int rc = layer_gate(b, c, gates[size_t(l) * nc + c]);
      if (rc) return rc;
    }
  // launch i holds every circuit's i-th block; circuits are independent, so a circuit whose gates
  // composed into fewer blocks simply has no operation in the later launches
  std::vector<int32_t> cursor(nc, 0);
  std::vector<BatchOp> ops(nc);
  for (;;) {
    bool any = false;
    for (uint32_t c = 0; c < nc; ++c) {
      next_block(b, c, gates, nlayers, W, &cursor[c], &ops[c]);
      any = any || ops[c].k != 0;
    }
    if (!any) break;
    int rc = b->prec == QD_C128 ? apply_layer_t<double>(b, ops) : apply_layer_t<float>(b, ops);
    if (rc) return rc;
  }
  return QD_OK;
}

int qd_batch_capture(qd_batch* b, int32_t on) {
  if (!b) return fail(QD_EINVAL, "null batch");
  if (on) {
    free_graph(b);
    QD_HIP(hipGraphCreate(&b->graph, 0));
    b->capturing = true;
    return QD_OK;
  }
  if (!b->capturing) return fail(QD_EINVAL, "no recording in progress");
  b->capturing = false;
  QD_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return QD_OK;
}

int qd_batch_replay(qd_batch* b) {
  if (!b) return fail(QD_EINVAL, "null batch");
  if (!b->exec) return fail(QD_EINVAL, "no recorded graph");
  QD_HIP(hipGraphLaunch(b->exec, b->stream));
  return QD_OK;
}

int qd_batch_download(const qd_batch* b, void* host, int64_t total) {
  if (!b || !host) return fail(QD_EINVAL, "null argument");
  if (total != b->total) return fail(QD_EDIM, "amplitude count differs from the arena size");
  QD_HIP(hipMemcpyAsync(host, b->arena, size_t(total) * amp_bytes(b->prec), hipMemcpyDeviceToHost, b->stream));
  QD_HIP(hipStreamSynchronize(b->stream));
  return QD_OK;
}

int qd_batch_autotune(qd_batch* b, const qd_gate* gates) {
  if (!b || !gates) return fail(QD_EINVAL, "null argument");
  if (b->capturing) return fail(QD_EINVAL, "cannot tune while recording");
  // the arena is saved and restored around the timed layers
  const size_t bytes = size_t(b->total) * amp_bytes(b->prec);
  void* save = nullptr;
  QD_HIP(hipMalloc(&save, bytes));
  hipError_t e = hipMemcpyAsync(save, b->arena, bytes, hipMemcpyDeviceToDevice, b->stream);
  TuneParams& tp = tune();
  const int old_block = tp.batch_block, old_spt = tp.batch_spt, old_wpc = tp.batch_wpc;
  int best_block = old_block, best_spt = old_spt, best_wpc = old_wpc, rc = QD_OK;
  float best = 1e30f;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (int blk : {128, 256})
    for (int spt : {2, 4, 8})
      for (int wpc : {8, 32, 64}) {
      if (e != hipSuccess || rc) break;
      tp.batch_block = blk;
      tp.batch_spt = spt;
      tp.batch_wpc = wpc;
      rc = qd_batch_apply_layer(b, gates);  // warm-up
      if (!rc) e = hipEventRecord(e0, b->stream);
      for (int i = 0; i < 3 && !rc && e == hipSuccess; ++i) rc = qd_batch_apply_layer(b, gates);
      if (!rc && e == hipSuccess) e = hipEventRecord(e1, b->stream);
      if (!rc && e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (!rc && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (!rc && e == hipSuccess && ms < best) {
        best = ms;
        best_block = blk;
        best_spt = spt;
        best_wpc = wpc;
      }
    }
  tp.batch_block = (rc || e != hipSuccess) ? old_block : best_block;
  tp.batch_spt = (rc || e != hipSuccess) ? old_spt : best_spt;
  tp.batch_wpc = (rc || e != hipSuccess) ? old_wpc : best_wpc;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  hipError_t e2 = hipMemcpyAsync(b->arena, save, bytes, hipMemcpyDeviceToDevice, b->stream);
  if (e2 == hipSuccess) e2 = hipStreamSynchronize(b->stream);
  (void)hipFree(save);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e, "batch autotune");
  if (e2 != hipSuccess) return hip_fail(e2, "batch autotune restore");
  return QD_OK;
}

}  // extern "C"

namespace qd {
// Amplitude updates per operation key of the blocks the layers form at fusion width W (host only).
static void key_shares(const qd_batch* b, const qd_gate* gates, int32_t nlayers, int W, double* share) {
  const uint32_t nc = uint32_t(b->regs.size());
  double tot = 0.0;
  for (int k = 0; k < QD_BATCH_KEYS; ++k) share[k] = 0.0;
  for (uint32_t c = 0; c < nc; ++c) {
    const Register& r = b->regs[c];
    int32_t cursor = 0;
    for (;;) {
      BatchOp o;
      next_block(b, c, gates, nlayers, W, &cursor, &o);
      if (o.k == 0) break;
      int dT = 1;
      int64_t smin = INT64_MAX;
      for (int j = 0; j < o.k; ++j) {
        dT *= r.dims[o.t[j]];
        smin = std::min<int64_t>(smin, r.strides[o.t[j]]);
      }
      const double upd = double(r.D) / (o.m == 1 ? double(r.dims[o.c]) : 1.0);
      share[batch_key(!o.members.empty(), dT, smin)] += upd;
      tot += upd;
    }
  }
  for (int k = 0; k < QD_BATCH_KEYS; ++k) share[k] = tot > 0.0 ? share[k] / tot : 0.0;
}

// Record the layers at fusion width w into the batch's graph, replay it once, then time two replays.
static int time_layers(qd_batch* b, const qd_gate* gates, int32_t nlayers, int w, hipEvent_t e0, hipEvent_t e1,
                       float* ms, hipError_t* e) {
  int rc = qd_batch_capture(b, 1);
  if (!rc) rc = qd_batch_apply_layers(b, gates, nlayers, w);
  if (b->capturing) {
    const int rc2 = qd_batch_capture(b, 0);
    if (!rc) rc = rc2;
  }
  if (!rc) rc = qd_batch_replay(b);   // warm-up
  if (!rc) *e = hipEventRecord(e0, b->stream);
  for (int i = 0; i < 2 && !rc && *e == hipSuccess; ++i) rc = qd_batch_replay(b);
  if (!rc && *e == hipSuccess) *e = hipEventRecord(e1, b->stream);
  if (!rc && *e == hipSuccess) *e = hipEventSynchronize(e1);
  if (!rc && *e == hipSuccess) *e = hipEventElapsedTime(ms, e0, e1);
  return rc;
}
}  // namespace qd

extern "C" {

int qd_batch_autotune_layers(qd_batch* b, const qd_gate* gates, int32_t nlayers) {
  if (!b || !gates || nlayers < 1) return fail(QD_EINVAL, "null argument or no layers");
  if (b->capturing) return fail(QD_EINVAL, "cannot tune while recording");
  const size_t bytes = size_t(b->total) * amp_bytes(b->prec);
  void* save = nullptr;
  QD_HIP(hipMalloc(&save, bytes));
  hipError_t e = hipMemcpyAsync(save, b->arena, bytes, hipMemcpyDeviceToDevice, b->stream);
  // each width is recorded into a graph of the tuner's own (the composition on the host happens
  // while recording, outside the timed replays); the caller's recorded graph is put aside meanwhile
  qd_batch mine;
  swap_graphs(b, &mine);
  TuneParams& tp = tune();
  const int old = tp.batch_fuse;
  int best_w = old, rc = QD_OK;
  float best = 1e30f;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (int w : {1, 2, 3, 4, 6, 8}) {
    if (rc || e != hipSuccess) break;
    float ms = 0.f;
    rc = time_layers(b, gates, nlayers, w, e0, e1, &ms, &e);
    if (!rc && e == hipSuccess && ms < best) {
      best = ms;
      best_w = w;
    }
  }
  tp.batch_fuse = (rc || e != hipSuccess) ? old : best_w;
  // then, at that width, slices per thread of the two wide slice classes in turn (0: the rule)
  for (int* knob : {&tp.batch_spt_mid, &tp.batch_spt_wide}) {
    const int keep = *knob;
    int best_v = keep;
    for (int v : {0, 1, 2, 4, 8}) {
      if (rc || e != hipSuccess || v == keep) continue;
      *knob = v;
      float ms = 0.f;
      rc = time_layers(b, gates, nlayers, best_w, e0, e1, &ms, &e);
      if (!rc && e == hipSuccess && ms < best) {
        best = ms;
        best_v = v;
      }
    }
    *knob = (rc || e != hipSuccess) ? keep : best_v;
  }
  // then each operation key that carries at least 3% of the amplitude updates at that width, in
  // decreasing share (a change must gain 1%: keys a workload lacks stay as they are)
  {
    double share[QD_BATCH_KEYS];
    key_shares(b, gates, nlayers, best_w, share);
    int order[QD_BATCH_KEYS];
    for (int k = 0; k < QD_BATCH_KEYS; ++k) order[k] = k;
    std::sort(order, order + QD_BATCH_KEYS, [&](int x, int y) { return share[x] > share[y]; });
    for (int k : order) {
      if (share[k] < 0.03) break;
      const int keep = tp.batch_spt_key[k];
      int best_v = keep;
      for (int v : {0, 1, 2, 4, 8}) {
        if (rc || e != hipSuccess || v == keep) continue;
        tp.batch_spt_key[k] = v;
        float ms = 0.f;
        rc = time_layers(b, gates, nlayers, best_w, e0, e1, &ms, &e);
        if (!rc && e == hipSuccess && ms < 0.99f * best) {
          best = ms;
          best_v = v;
        }
      }
      tp.batch_spt_key[k] = (rc || e != hipSuccess) ? keep : best_v;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  hipError_t e2 = hipMemcpyAsync(b->arena, save, bytes, hipMemcpyDeviceToDevice, b->stream);
  if (e2 == hipSuccess) e2 = hipStreamSynchronize(b->stream);
  free_graph(b);
  swap_graphs(b, &mine);
  (void)hipFree(save);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e, "batch fusion autotune");
  if (e2 != hipSuccess) return hip_fail(e2, "batch fusion autotune restore");
  return QD_OK;
}

int qd_batch_compose_ms(qd_batch* b, double* ms) {
  if (!b || !ms) return fail(QD_EINVAL, "null argument");
  double tot = b->compose_ms;
  b->compose_ms = 0.0;
  hipError_t err = hipSuccess;
  for (auto& ev : b->compose_ev) {
    float t = 0.f;
    if (err == hipSuccess) err = hipEventSynchronize(ev.second);
    if (err == hipSuccess) err = hipEventElapsedTime(&t, ev.first, ev.second);
    tot += t;
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  b->compose_ev.clear();
  if (err != hipSuccess) return hip_fail(err, "batch composition timing");
  *ms = tot;
  return QD_OK;
}

void qd_batch_free(qd_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  for (auto& ev : b->compose_ev) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  free_graph(b);
  if (b->arena) (void)hipFree(b->arena);
  if (b->offs_dev) (void)hipFree(b->offs_dev);
  ring_free(&b->ring);
  delete b;
}

}  // extern "C"
