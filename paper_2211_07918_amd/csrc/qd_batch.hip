// Batched circuits: many independent registers of different sizes in one device arena, advanced
// one gate layer (the paper's Moment, Sec. 3.5) at a time by ONE persistent launch per layer.
//
// A layer holds at most one single-target gate (optionally with one control) per circuit. The host
// turns it into a descriptor per circuit (arena offset, slice map, U) and a prefix sum of work
// tiles (a tile is `block x spt` consecutive slices of one circuit). Each workgroup walks a
// contiguous range of the global tile list: one binary search to find its first circuit, then it
// steps forward, so heterogeneous registers and gates share one launch with divergence only
// between tiles, never inside a wavefront. Layers can be recorded into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "qd_internal.h"

namespace qd {

constexpr int kBatchMaxDim = 8;
constexpr int kBatchGroups = 3;

struct BatchDesc {
  int64_t off;                      // arena offset of the circuit's state (amplitudes)
  int64_t base;                     // control offset inside the state
  int64_t st;                       // target stride
  uint32_t nwork;                   // active slices
  uint32_t tile0;                   // first global tile of this circuit
  int32_t dt;                       // target dimension, 0 = no gate in this layer
  int32_t ng;                       // slice-map groups
  uint32_t uoff;                    // offset of U in the layer's value pool
  uint32_t pad;
  uint32_t gdim[kBatchGroups];
  uint32_t pad2;
  Magic32 gmag[kBatchGroups];
  int64_t gstride[kBatchGroups];
};

template <typename R>
struct BatchArgs {
  R* arena;
  const BatchDesc* desc;
  const R* upool;
  uint32_t ncirc;
  uint32_t ntiles;
  uint32_t spt;
};

template <typename R> struct CxB;
template <> struct CxB<double> { using T = double2; };
template <> struct CxB<float> { using T = float2; };

__device__ __forceinline__ int64_t bd_offset(const BatchDesc& d, uint32_t idx) {
  int64_t off = d.base;
  uint32_t rem = idx;
#pragma unroll
  for (int g = 0; g < kBatchGroups; ++g) {
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
// the kernel stays that of about 16 amplitudes whatever the gate's dimension)
constexpr int kBatchMaxSpt = 8;

#ifndef QD_BATCH_LD
#define QD_BATCH_LD(p) (*(p))
#define QD_BATCH_ST(p, v) (*(p) = (v))
#endif

template <typename R, int DT>
__device__ __forceinline__ void batch_tile(const BatchArgs<R>& a, const BatchDesc& d, uint32_t j0, uint32_t j1) {
  using C = typename CxB<R>::T;
  constexpr int KB = (16 / DT) < 1 ? 1 : ((16 / DT) > kBatchMaxSpt ? kBatchMaxSpt : (16 / DT));
  C* psi = reinterpret_cast<C*>(a.arena) + d.off;
  const R* U = a.upool + d.uoff;
  for (int k0 = 0; k0 < int(a.spt); k0 += KB) {
    int64_t b[KB];
    C x[KB][DT];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const uint32_t j = j0 + threadIdx.x + uint32_t(k0 + k) * blockDim.x;
      b[k] = (k0 + k < int(a.spt) && j < j1) ? bd_offset(d, j) : -1;
      if (b[k] >= 0) {
#pragma unroll
        for (int y = 0; y < DT; ++y) x[k][y] = QD_BATCH_LD(psi + (b[k] + y * d.st));
      }
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      if (b[k] < 0) continue;
#pragma unroll
      for (int r = 0; r < DT; ++r) {
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
        QD_BATCH_ST(psi + (b[k] + r * d.st), yv);
      }
    }
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_batch_layer(BatchArgs<R> a) {
  const uint32_t per = (a.ntiles + gridDim.x - 1) / gridDim.x;
  const uint32_t t0 = blockIdx.x * per;
  const uint32_t t1 = min(a.ntiles, t0 + per);
  if (t0 >= t1) return;
  // first circuit whose tile range holds t0: last c with tile0 <= t0 among circuits with work
  uint32_t lo = 0, hi = a.ncirc;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a.desc[mid].tile0 <= t0) lo = mid;
    else hi = mid;
  }
  uint32_t c = lo;
  const uint32_t tile_slices = blockDim.x * a.spt;
  for (uint32_t t = t0; t < t1; ++t) {
    while (c + 1 < a.ncirc && a.desc[c + 1].tile0 <= t) ++c;
    const BatchDesc& d = a.desc[c];
    const uint32_t j0 = (t - d.tile0) * tile_slices;
    const uint32_t j1 = min(d.nwork, j0 + tile_slices);
    switch (d.dt) {
      case 2: batch_tile<R, 2>(a, d, j0, j1); break;
      case 3: batch_tile<R, 3>(a, d, j0, j1); break;
      case 4: batch_tile<R, 4>(a, d, j0, j1); break;
      case 5: batch_tile<R, 5>(a, d, j0, j1); break;
      case 6: batch_tile<R, 6>(a, d, j0, j1); break;
      case 7: batch_tile<R, 7>(a, d, j0, j1); break;
      case 8: batch_tile<R, 8>(a, d, j0, j1); break;
      default: break;
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
};

namespace qd {

template <typename R>
static void* batch_kernel_ptr() {
  return reinterpret_cast<void*>(k_batch_layer<R>);
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

// Host: descriptors and U pool of one layer; returns the total tile count.
template <typename R>
static int build_layer(qd_batch* b, const qd_gate* gates, std::vector<BatchDesc>* desc, std::vector<R>* pool,
                       uint32_t* ntiles) {
  const uint32_t nc = uint32_t(b->regs.size());
  const TuneParams& tp = tune();
  const uint64_t tile_slices = uint64_t(tp.batch_block) * tp.batch_spt;
  desc->assign(nc, BatchDesc{});
  pool->clear();
  uint64_t tiles = 0;
  for (uint32_t c = 0; c < nc; ++c) {
    const Register& r = b->regs[c];
    BatchDesc& d = (*desc)[c];
    d.off = b->offs[c];
    d.tile0 = uint32_t(tiles);
    const qd_gate& G = gates[c];
    if (G.k == 0) continue;
    if (G.k != 1 || G.m > 1) return fail(QD_EINVAL, "batched layers take one target and at most one control (circuit " + std::to_string(c) + ")");
    int rc = validate_gate(r, G.targets, G.k, G.controls, G.control_values, G.m, G.U, 0);
    if (rc) return fail(rc, "circuit " + std::to_string(c) + ": " + qd_last_error());
    const int t = G.targets[0];
    const int dt = r.dims[t];
    if (dt > kBatchMaxDim) return fail(QD_EINVAL, "batched layers support target dimensions up to 8");
    int role[QD_MAX_QUDITS] = {};
    role[t] = 1;
    int64_t base = 0;
    if (G.m == 1) {
      role[G.controls[0]] = 1;
      base = int64_t(G.control_values[0]) * r.strides[G.controls[0]];
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
    d.st = r.strides[t];
    d.dt = dt;
    d.nwork = uint32_t(nwork);
    d.uoff = uint32_t(pool->size());
    for (int i = 0; i < 2 * dt * dt; ++i) pool->push_back(R(G.U[i]));
    tiles += (nwork + tile_slices - 1) / tile_slices;
    if (tiles > 0xFFFFFFF0ull) return fail(QD_EOVERFLOW, "too many tiles in one layer");
  }
  *ntiles = uint32_t(tiles);
  return QD_OK;
}

template <typename R>
static int apply_layer_t(qd_batch* b, const qd_gate* gates) {
  std::vector<BatchDesc> desc;
  std::vector<R> pool;
  uint32_t ntiles = 0;
  int rc = build_layer<R>(b, gates, &desc, &pool, &ntiles);
  if (rc) return rc;
  const size_t dbytes = desc.size() * sizeof(BatchDesc);
  const size_t pbytes = std::max<size_t>(pool.size(), 1) * sizeof(R);
  const size_t dpad = (dbytes + 255) / 256 * 256;
  std::vector<unsigned char> blob(dpad + pbytes, 0);
  std::memcpy(blob.data(), desc.data(), dbytes);
  if (!pool.empty()) std::memcpy(blob.data() + dpad, pool.data(), pool.size() * sizeof(R));
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
  a.spt = uint32_t(tp.batch_spt);
  if (!b->capturing) {
    if (ntiles == 0) return QD_OK;
    void* dev_blob = nullptr;
    rc = ring_push_stream(&b->ring, b->stream, blob.data(), blob.size(), &dev_blob);
    if (rc) return rc;
    a.desc = reinterpret_cast<const BatchDesc*>(dev_blob);
    a.upool = reinterpret_cast<const R*>(static_cast<unsigned char*>(dev_blob) + dpad);
    hipLaunchKernelGGL((k_batch_layer<R>), dim3(grid), dim3(tp.batch_block), 0, b->stream, a);
    QD_HIP(hipGetLastError());
    return QD_OK;
  }
  // recording: the layer's parameters live in their own device buffer for the graph's lifetime
  void* buf = nullptr;
  QD_HIP(hipMalloc(&buf, blob.size()));
  b->layer_bufs.push_back(buf);
  QD_HIP(hipMemcpy(buf, blob.data(), blob.size(), hipMemcpyHostToDevice));
  if (ntiles == 0) return QD_OK;
  a.desc = reinterpret_cast<const BatchDesc*>(buf);
  a.upool = reinterpret_cast<const R*>(static_cast<unsigned char*>(buf) + dpad);
  b->layer_args.emplace_back(sizeof(a));
  std::memcpy(b->layer_args.back().data(), &a, sizeof(a));
  void* kargs[1] = {b->layer_args.back().data()};
  hipKernelNodeParams kp{};
  kp.blockDim = dim3(tp.batch_block);
  kp.gridDim = dim3(grid);
  kp.func = batch_kernel_ptr<R>();
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
  return b->prec == QD_C128 ? apply_layer_t<double>(b, gates) : apply_layer_t<float>(b, gates);
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

void qd_batch_free(qd_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  free_graph(b);
  if (b->arena) (void)hipFree(b->arena);
  if (b->offs_dev) (void)hipFree(b->offs_dev);
  ring_free(&b->ring);
  delete b;
}

}  // extern "C"
