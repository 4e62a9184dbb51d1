// Gate fusion: the paper evaluates a circuit by multiplying the operators of all Moments into one
// D x D matrix (Sec. 3.6). qd_fuse bounds that idea: consecutive gates are grouped while the union
// of their qudits (a window) spans at most max_block_dim basis states, and each group is
// multiplied out into one B x B block in FP64 on the GPU. The blocks are then applied to the state
// like a dense gate on the window, in FP64 or on the matrix cores in FP32 / split BF16.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "qd_fused.h"

namespace qd {

// ------------------------------------------------------------------------------------------ planner
// A block starts at the first gate not yet placed. Later gates join it while the window (union of
// the members' targets and controls) spans at most max_block basis states. A gate that does not
// join is skipped, and its qudits become blocked: a later gate may still join only if it commutes
// with every skipped gate it would move ahead of. Two gates commute exactly when their qudits are
// disjoint, or when both are diagonal (controlled phases, Z_d). Members keep their circuit order,
// so each block is an exact product of Moment operators up to such commutations.
int plan_fusion(const Register& r, const qd_gate* gates, int32_t g, int32_t max_block,
                std::vector<int32_t>* block_of, std::vector<FusedBlockInfo>* blocks) {
  if (g < 0 || (g > 0 && !gates)) return fail(QD_EINVAL, "bad gate list");
  if (max_block < 2 || max_block > QD_MAX_FUSED_DIM) return fail(QD_EINVAL, "max_block_dim must be 2..128");
  block_of->assign(size_t(g), -1);
  blocks->clear();
  std::vector<uint64_t> mask(size_t(g), 0);    // qudit set of each gate (n <= 64)
  std::vector<char> diag(size_t(g), 0);
  for (int i = 0; i < g; ++i) {
    const qd_gate& G = gates[i];
    if (G.k < 1 || !G.targets || G.m < 0 || (G.m > 0 && (!G.controls || !G.control_values)))
      return fail(QD_EINVAL, "malformed gate " + std::to_string(i));
    int64_t own = 1;
    for (int j = 0; j < G.k + G.m; ++j) {
      const int q = j < G.k ? G.targets[j] : G.controls[j - G.k];
      if (q < 0 || q >= r.n) return fail(QD_EINVAL, "qudit out of range in gate " + std::to_string(i));
      if (!(mask[i] >> q & 1)) own *= r.dims[q];
      mask[i] |= uint64_t(1) << q;
    }
    if (own > max_block) return fail(QD_EDIM, "gate " + std::to_string(i) + " spans more than max_block_dim");
    int64_t dT = 1;
    for (int j = 0; j < G.k; ++j) dT *= r.dims[G.targets[j]];
    diag[i] = G.U && classify(G.U, int(dT)) == QD_CLASS_DIAGONAL;
  }
  auto span = [&](uint64_t m) {
    int64_t p = 1;
    for (int q = 0; q < r.n; ++q)
      if (m >> q & 1) p *= r.dims[q];
    return p;
  };
  const uint64_t all = r.n == 64 ? ~uint64_t(0) : ((uint64_t(1) << r.n) - 1);
  int first = 0;
  while (first < g) {
    FusedBlockInfo nb{};
    const int bidx = int(blocks->size());
    // qudits of skipped non-diagonal gates (block everything) and of skipped diagonal gates
    // (block only non-diagonal gates)
    uint64_t win = mask[first], blocked = 0, blocked_diag = 0;
    nb.members.push_back(first);
    (*block_of)[first] = bidx;
    for (int i = first + 1; i < g; ++i) {
      if ((*block_of)[i] >= 0) continue;
      const bool passes = !(mask[i] & blocked) && (diag[i] || !(mask[i] & blocked_diag));
      if (passes && span(win | mask[i]) <= max_block) {
        win |= mask[i];
        nb.members.push_back(i);
        (*block_of)[i] = bidx;
        continue;
      }
      if (diag[i]) blocked_diag |= mask[i];
      else blocked |= mask[i];
      if ((blocked | win) == all && (blocked & win) == win) break;  // nothing can join any more
    }
    nb.k = 0;
    for (int q = 0; q < r.n; ++q)
      if (win >> q & 1) nb.window[nb.k++] = q;
    nb.B = int32_t(span(win));
    nb.first_gate = nb.members.front();
    nb.ngates = int32_t(nb.members.size());
    blocks->push_back(nb);
    while (first < g && (*block_of)[first] >= 0) ++first;
  }
  return QD_OK;
}

// ------------------------------------------------------------------------------------------ casts
// Real embedding of a complex B x B block U with interleaved rows/columns: row 2y'+c', column
// 2y+c carries the 2x2 real block [[Re u, -Im u], [Im u, Re u]] of u = U[y', y]. Padded with zeros
// to Kp x Kp, row-major FP32, plus the BF16 split hi = bf16(a), lo = bf16(a - hi).
__global__ __launch_bounds__(256) void k_embed(const double* __restrict__ U, int B, int Kp, float* __restrict__ a32,
                                               __hip_bfloat16* __restrict__ ahi, __hip_bfloat16* __restrict__ alo) {
  const int n = Kp * Kp;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int row = e / Kp, col = e - row * Kp;
    double v = 0.0;
    if (row < 2 * B && col < 2 * B) {
      const int yr = row >> 1, cr = row & 1, yc = col >> 1, cc = col & 1;
      const double ur = U[2 * (size_t(yr) * B + yc)], ui = U[2 * (size_t(yr) * B + yc) + 1];
      v = cr == 0 ? (cc == 0 ? ur : -ui) : (cc == 0 ? ui : ur);
    }
    const float f = float(v);
    a32[e] = f;
    const __hip_bfloat16 h = __float2bfloat16(f);
    ahi[e] = h;
    alo[e] = __float2bfloat16(f - __bfloat162float(h));
  }
}

int embed_block(qd_fused* f, int b) {
  FusedBlockDev& d = f->dev[b];
  const int n = d.Kp * d.Kp;
  hipLaunchKernelGGL(k_embed, dim3(std::min(1024, (n + 255) / 256)), dim3(256), 0, f->stream, d.u64, d.info.B, d.Kp,
                     d.a32, d.ahi, d.alo);
  QD_HIP(hipGetLastError());
  return QD_OK;
}

static int pad_k(int B) { return fused_kpad(B); }

}  // namespace qd

using namespace qd;

extern "C" {

int qd_fuse_plan(const int32_t* dims, int32_t n, const qd_gate* gates, int32_t g, int32_t max_block_dim,
                 int32_t* block_of_gate, int32_t* nblocks) {
  if (!block_of_gate || !nblocks) return fail(QD_EINVAL, "null output");
  Register r;
  int rc = make_register(dims, n, &r);
  if (rc) return rc;
  std::vector<int32_t> bo;
  std::vector<FusedBlockInfo> blocks;
  rc = plan_fusion(r, gates, g, max_block_dim, &bo, &blocks);
  if (rc) return rc;
  for (int i = 0; i < g; ++i) block_of_gate[i] = bo[i];
  *nblocks = int32_t(blocks.size());
  return QD_OK;
}

int qd_fuse(const int32_t* dims, int32_t n, const qd_gate* gates, int32_t g, int32_t max_block_dim,
            void* hip_stream, qd_fused** out) {
  if (!out) return fail(QD_EINVAL, "null output handle");
  Register r;
  int rc = make_register(dims, n, &r);
  if (rc) return rc;
  for (int i = 0; i < g; ++i) {
    if (!gates) return fail(QD_EINVAL, "null gate list");
    rc = validate_gate(r, gates[i].targets, gates[i].k, gates[i].controls, gates[i].control_values, gates[i].m,
                       gates[i].U, 0);
    if (rc) return fail(rc, "gate " + std::to_string(i) + ": " + qd_last_error());
  }
  std::vector<int32_t> bo;
  std::vector<FusedBlockInfo> blocks;
  if (max_block_dim == 0) {
    // fusion width from a cost model: matrix-core time vs HBM time per block
    const double F = 40e12, H = 5e12, D = double(r.D);
    double best = 1e300;
    for (int cand : {16, 27, 32, 36, 48, 64, 81, 96, 128}) {
      std::vector<int32_t> cbo;
      std::vector<FusedBlockInfo> cbl;
      if (plan_fusion(r, gates, g, cand, &cbo, &cbl) != QD_OK) continue;
      double cost = 0.0;
      for (const auto& bl : cbl) cost += std::max(8.0 * bl.B * D / F, 16.0 * D / H);
      if (cost < best) {
        best = cost;
        bo.swap(cbo);
        blocks.swap(cbl);
      }
    }
    if (best == 1e300) return fail(QD_EDIM, "no fusion width fits the circuit's gates");
  } else {
    rc = plan_fusion(r, gates, g, max_block_dim, &bo, &blocks);
    if (rc) return rc;
  }

  auto* f = new qd_fused();
  f->reg = r;
  f->stream = (hipStream_t)hip_stream;
  f->dev.resize(blocks.size());
  auto cleanup = [&](int code) {
    qd_fused_free(f);
    return code;
  };
  for (size_t b = 0; b < blocks.size(); ++b) {
    FusedBlockDev& d = f->dev[b];
    d.info = blocks[b];
    const int B = d.info.B;
    d.Kp = pad_k(B);
    hipError_t e = hipMalloc((void**)&d.u64, sizeof(double) * 2 * size_t(B) * B);
    if (e == hipSuccess) e = hipMalloc((void**)&d.a32, sizeof(float) * size_t(d.Kp) * d.Kp);
    if (e == hipSuccess) e = hipMalloc((void**)&d.ahi, sizeof(__hip_bfloat16) * size_t(d.Kp) * d.Kp);
    if (e == hipSuccess) e = hipMalloc((void**)&d.alo, sizeof(__hip_bfloat16) * size_t(d.Kp) * d.Kp);
    if (e != hipSuccess) return cleanup(hip_fail(e, "fused block allocation"));

    // The block is built by applying its gates, embedded in the window register, to the
    // identity: a register with the window's dims plus one extra lowest digit of size B holding
    // the column index, so M <- E_g M for every column at once (FP64, the plain gate kernels).
    int32_t wdims[QD_MAX_QUDITS + 1];
    int pos[QD_MAX_QUDITS];
    for (int j = 0; j < d.info.k; ++j) {
      wdims[j] = r.dims[d.info.window[j]];
      pos[d.info.window[j]] = j;
    }
    wdims[d.info.k] = B;
    qd_state tmp;
    rc = make_register(wdims, d.info.k + 1, &tmp.reg);
    if (rc) return cleanup(rc);
    tmp.prec = QD_C128;
    tmp.data = d.u64;
    tmp.owned = false;
    tmp.stream = f->stream;
    // identity: amplitude (row, col) = delta(row, col) at flat index row * B + col
    std::vector<double> eye(2 * size_t(B) * B, 0.0);
    for (int y = 0; y < B; ++y) eye[2 * (size_t(y) * B + y)] = 1.0;
    e = hipMemcpyAsync(d.u64, eye.data(), eye.size() * sizeof(double), hipMemcpyHostToDevice, f->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) return cleanup(hip_fail(e, "fused block init"));
    for (int i : d.info.members) {
      const qd_gate& G = gates[i];
      int32_t t[QD_MAX_QUDITS], c[QD_MAX_QUDITS];
      for (int j = 0; j < G.k; ++j) t[j] = pos[G.targets[j]];
      for (int j = 0; j < G.m; ++j) c[j] = pos[G.controls[j]];
      GatePlan p;
      make_plan(tmp.reg, t, G.k, c, G.control_values, G.m, G.U, &p);
      rc = launch_gate(&tmp, p);
      if (rc) {
        ring_free(&tmp.ring);
        return cleanup(rc);
      }
    }
    e = hipStreamSynchronize(f->stream);
    ring_free(&tmp.ring);
    if (e != hipSuccess) return cleanup(hip_fail(e, "fused block build"));
    rc = embed_block(f, int(b));
    if (rc) return cleanup(rc);
    if (r.D <= int64_t(0xFFFFFFFFll)) {
      rc = fused_geometry(r, &d);
      if (rc) return cleanup(rc);
    }
    d.host64.resize(2 * size_t(B) * B);
  }
  // host copies of the FP64 blocks for the FP64 apply path
  for (auto& d : f->dev) {
    hipError_t e = hipMemcpyAsync(d.host64.data(), d.u64, d.host64.size() * sizeof(double), hipMemcpyDeviceToHost,
                                  f->stream);
    if (e != hipSuccess) return cleanup(hip_fail(e, "fused block download"));
  }
  hipError_t e = hipStreamSynchronize(f->stream);
  if (e != hipSuccess) return cleanup(hip_fail(e, "qd_fuse"));
  *out = f;
  return QD_OK;
}

int qd_fused_count(const qd_fused* f, int32_t* nblocks) {
  if (!f || !nblocks) return fail(QD_EINVAL, "null argument");
  *nblocks = int32_t(f->dev.size());
  return QD_OK;
}

int qd_fused_block_info(const qd_fused* f, int32_t b, int32_t* k, int32_t* window, int32_t* B, int32_t* first,
                        int32_t* ng) {
  if (!f) return fail(QD_EINVAL, "null handle");
  if (b < 0 || b >= int32_t(f->dev.size())) return fail(QD_EINVAL, "block index out of range");
  const FusedBlockInfo& i = f->dev[b].info;
  if (k) *k = i.k;
  if (window)
    for (int j = 0; j < i.k; ++j) window[j] = i.window[j];
  if (B) *B = i.B;
  if (first) *first = i.first_gate;
  if (ng) *ng = i.ngates;
  return QD_OK;
}

int qd_fused_block_gates(const qd_fused* f, int32_t b, int32_t* gates_out) {
  if (!f || !gates_out) return fail(QD_EINVAL, "null argument");
  if (b < 0 || b >= int32_t(f->dev.size())) return fail(QD_EINVAL, "block index out of range");
  const FusedBlockInfo& i = f->dev[b].info;
  for (size_t j = 0; j < i.members.size(); ++j) gates_out[j] = i.members[j];
  return QD_OK;
}

int qd_fused_download_block(const qd_fused* f, int32_t b, double* out) {
  if (!f || !out) return fail(QD_EINVAL, "null argument");
  if (b < 0 || b >= int32_t(f->dev.size())) return fail(QD_EINVAL, "block index out of range");
  const auto& d = f->dev[b];
  std::memcpy(out, d.host64.data(), d.host64.size() * sizeof(double));
  return QD_OK;
}

int qd_apply_fused(qd_state* s, const qd_fused* f, int32_t mode_flags) {
  if (!s || !f) return fail(QD_EINVAL, "null argument");
  if (mode_flags & ~int32_t(0xFF | QD_FUSED_RENORMALIZE)) return fail(QD_EINVAL, "unknown mode flag");
  set_last_kernel("");
  const int32_t mode = mode_flags & 0xFF;
  const bool renorm = (mode_flags & QD_FUSED_RENORMALIZE) != 0;
  if (s->reg.n != f->reg.n) return fail(QD_EDIM, "register differs from the fused circuit's");
  for (int i = 0; i < s->reg.n; ++i)
    if (s->reg.dims[i] != f->reg.dims[i]) return fail(QD_EDIM, "register differs from the fused circuit's");
  if (mode == QD_MODE_FP64_PLAIN) {
    if (s->prec != QD_C128) return fail(QD_EDIM, "FP64 mode needs a complex128 state");
    for (const auto& d : f->dev) {
      GatePlan p;
      make_plan(s->reg, d.info.window, d.info.k, nullptr, nullptr, 0, d.host64.data(), &p);
      int rc = launch_gate(s, p);
      if (rc) return rc;
    }
    return renorm ? normalize_on_device(s) : QD_OK;
  }
  if (mode != QD_MODE_FP32_MFMA && mode != QD_MODE_BF16X3_MFMA) return fail(QD_EINVAL, "unknown mode");
  if (s->prec != QD_C64) return fail(QD_EDIM, "matrix-core modes need a complex64 state");
  if (s->reg.D > int64_t(0xFFFFFFFFll)) return fail(QD_EOVERFLOW, "matrix-core path needs D < 2^32");
  for (size_t b = 0; b < f->dev.size(); ++b) {
    int rc = launch_fused_block(s, f, int(b), mode);
    if (rc) return rc;
  }
  return renorm ? normalize_on_device(s) : QD_OK;
}

void qd_fused_free(qd_fused* f) {
  if (!f) return;
  (void)hipStreamSynchronize(f->stream);
  for (auto& d : f->dev) {
    if (d.u64) (void)hipFree(d.u64);
    if (d.a32) (void)hipFree(d.a32);
    if (d.ahi) (void)hipFree(d.ahi);
    if (d.alo) (void)hipFree(d.alo);
    if (d.tab_hoff) (void)hipFree(d.tab_hoff);
    if (d.tab_yh) (void)hipFree(d.tab_yh);
    if (d.tab_lmap) (void)hipFree(d.tab_lmap);
    if (d.tab_rowpos) (void)hipFree(d.tab_rowpos);
    if (d.tab_rowpos_odd) (void)hipFree(d.tab_rowpos_odd);
    if (d.tab_colpos) (void)hipFree(d.tab_colpos);
    if (d.tab_wrow) (void)hipFree(d.tab_wrow);
  }
  delete f;
}

}  // extern "C"
