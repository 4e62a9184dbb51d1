// Autotuner: tile shapes of the gate kernels per (precision, stride class of the gate's smallest
// target stride), chosen by timing every candidate with HIP events on a scratch state, plus the
// batched layer kernel's tile shape. The table is process-wide and can be saved to / loaded from
// a small JSON file (one entry per line).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "qd_internal.h"

namespace qd {

static TuneEntry g_table[2][kStrideBuckets];
static bool g_table_valid = false;

// Strides of 256 to 4095 amplitudes and larger ones are tuned apart: a direct-kernel shape chosen on
// a gate whose two planes lie megabytes apart can be several percent off for planes a few
// kilobytes apart, and the reverse.
int stride_bucket(int64_t s) {
  return s < 2 ? 0 : (s < 4 ? 1 : (s < 16 ? 2 : (s < 256 ? 3 : (s < 4096 ? 4 : 5))));
}

TuneEntry entry_for(int prec, int64_t min_stride) {
  const int b = stride_bucket(min_stride);
  const int p = prec == QD_C128 ? 0 : 1;
  if (g_table_valid && g_table[p][b].valid) return g_table[p][b];
  const TuneParams& tp = tune();
  TuneEntry e;
  e.valid = 1;
  e.tiled = min_stride < tp.run_min ? 1 : 0;
  e.block = e.tiled ? tp.tile_block : tp.direct_block;
  e.spt = tp.direct_spt;
  e.tile_elems = tp.tile_elems;
  return e;
}

void clear_tuned_table() { g_table_valid = false; }

// Time of one launch: the fastest of five rounds of two launches each, after a warm-up. Candidates
// a few percent apart are common (thread counts of the tile kernel, slices per thread), and noise
// only ever adds time, so the minimum over rounds separates them where one average would not.
static int time_gate(qd_state* s, const GatePlan& p, float* ms) {
  hipEvent_t e0, e1;
  QD_HIP(hipEventCreate(&e0));
  QD_HIP(hipEventCreate(&e1));
  int rc = launch_gate(s, p);  // warm-up (also compiles nothing: code objects are loaded)
  *ms = 1e30f;
  for (int round = 0; round < 5 && !rc; ++round) {
    float t = 0.f;
    hipError_t e = hipEventRecord(e0, s->stream);
    for (int i = 0; i < 2 && !rc && e == hipSuccess; ++i) rc = launch_gate(s, p);
    if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e != hipSuccess && !rc) rc = hip_fail(e, "autotune timing");
    if (!rc) *ms = std::min(*ms, t / 2.0f);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

static int write_table(const char* path) {
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(QD_EINVAL, std::string("cannot write ") + path);
  std::fprintf(f, "[\n");
  bool first = true;
  for (int p = 0; p < 2; ++p)
    for (int b = 0; b < kStrideBuckets; ++b) {
      const TuneEntry& e = g_table[p][b];
      if (!g_table_valid || !e.valid) continue;
      std::fprintf(f, "%s{\"prec\": %d, \"bucket\": %d, \"tiled\": %d, \"block\": %d, \"spt\": %d, \"tile_elems\": %d}",
                   first ? "" : ",\n", p, b, e.tiled, e.block, e.spt, e.tile_elems);
      first = false;
    }
  const TuneParams& tp = tune();
  std::fprintf(f,
               "%s{\"batch_block\": %d, \"batch_spt\": %d, \"batch_grid\": %d, \"batch_fuse\": %d, "
               "\"batch_spt_mid\": %d, \"batch_spt_wide\": %d}",
               first ? "" : ",\n", tp.batch_block, tp.batch_spt, tp.batch_wpc, tp.batch_fuse, tp.batch_spt_mid,
               tp.batch_spt_wide);
  // slices per thread of the batched kernel per operation key (0: inherited)
  static const char* gate_cls[2] = {"one gate", "composed"};
  static const char* slice_cls[3] = {"2-4", "5-9", "12-32"};
  static const char* stride_cls[2] = {"< 16", ">= 16"};
  for (int k = 0; k < QD_BATCH_KEYS; ++k)
    std::fprintf(f, ",\n{\"batch_key\": %d, \"gate\": \"%s\", \"d_T\": \"%s\", \"min_stride\": \"%s\", \"spt\": %d}", k,
                 gate_cls[k / 6], slice_cls[(k / 2) % 3], stride_cls[k % 2], tp.batch_spt_key[k]);
  std::fprintf(f, "\n]\n");
  std::fclose(f);
  return QD_OK;
}

}  // namespace qd

using namespace qd;

extern "C" {

int qd_autotune(qd_state* s, const char* path) {
  if (!s) return fail(QD_EINVAL, "null state");
  const int p = s->prec == QD_C128 ? 0 : 1;
  TuneEntry tuned[kStrideBuckets] = {};
  for (int b = 0; b < kStrideBuckets; ++b) {
    // a qudit of this stride class, preferring the largest radix
    int t = -1;
    for (int q = 0; q < s->reg.n; ++q)
      if (stride_bucket(s->reg.strides[q]) == b && (t < 0 || s->reg.dims[q] > s->reg.dims[t])) t = q;
    if (t < 0 || s->reg.dims[t] > kMaxInlineDense) continue;
    const int d = s->reg.dims[t];
    std::vector<double> U(2 * size_t(d) * d);
    int rc = qd_gate_matrix(QD_GATE_F, d, 0, U.data());
    if (rc) return rc;
    GatePlan plan;
    const int32_t tg[1] = {t};
    make_plan(s->reg, tg, 1, nullptr, nullptr, 0, U.data(), &plan);
    std::vector<TuneEntry> cands;
    for (int blk : {64, 128, 256})
      for (int spt : {1, 2, 4}) cands.push_back(TuneEntry{1, 0, blk, spt, 2048});
    for (int te : {512, 1024, 2048, 4096})
      for (int blk : {128, 256}) cands.push_back(TuneEntry{1, 1, blk, 1, te});
    float best = 1e30f;
    for (const TuneEntry& c : cands) {
      g_table[p][b] = c;
      g_table_valid = true;
      // a tiled candidate that cannot form a tile runs the direct kernel: skip it
      if (c.tiled) {
        TileGeom g;
        if (!tile_geometry(s->reg, plan, s->prec, &g)) continue;
      }
      float ms = 0.f;
      rc = time_gate(s, plan, &ms);
      if (rc) {
        g_table_valid = false;
        return rc;
      }
      if (ms < best) {
        best = ms;
        tuned[b] = c;
      }
    }
  }
  for (int b = 0; b < kStrideBuckets; ++b) g_table[p][b] = tuned[b];
  g_table_valid = true;
  if (path) return write_table(path);
  return QD_OK;
}

int qd_tune_load(const char* path) {
  if (!path) return fail(QD_EINVAL, "null path");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(QD_EINVAL, std::string("cannot read ") + path);
  TuneEntry tab[2][kStrideBuckets] = {};
  int batch_block = 0, batch_spt = 0, batch_grid = 0, batch_fuse = 0, spt_mid = 0, spt_wide = 0, n = 0;
  int key_spt[QD_BATCH_KEYS] = {};
  char line[512];
  while (std::fgets(line, sizeof(line), f)) {
    int p, b, tiled, block, spt, te, key;
    if (std::sscanf(line, " {\"batch_key\": %d,", &key) == 1) {
      const char* sp = std::strstr(line, "\"spt\": ");
      int v = -1;
      if (!sp || std::sscanf(sp, "\"spt\": %d", &v) != 1 || key < 0 || key >= QD_BATCH_KEYS ||
          (v != 0 && v != 1 && v != 2 && v != 4 && v != 8)) {
        std::fclose(f);
        return fail(QD_EINVAL, "batch key entry out of range");
      }
      key_spt[key] = v;
      ++n;
      continue;
    }
    if (std::sscanf(line, " {\"prec\": %d, \"bucket\": %d, \"tiled\": %d, \"block\": %d, \"spt\": %d, \"tile_elems\": %d}",
                    &p, &b, &tiled, &block, &spt, &te) == 6) {
      if (p < 0 || p > 1 || b < 0 || b >= kStrideBuckets || (block != 64 && block != 128 && block != 192 && block != 256) ||
          (spt != 1 && spt != 2 && spt != 4) || te < 256 || te > 4096) {
        std::fclose(f);
        return fail(QD_EINVAL, "tuning entry out of range");
      }
      tab[p][b] = TuneEntry{1, tiled ? 1 : 0, block, spt, te};
      ++n;
    } else if (std::sscanf(line,
                           " {\"batch_block\": %d, \"batch_spt\": %d, \"batch_grid\": %d, \"batch_fuse\": %d, "
                           "\"batch_spt_mid\": %d, \"batch_spt_wide\": %d}",
                           &batch_block, &batch_spt, &batch_grid, &batch_fuse, &spt_mid, &spt_wide) >= 2) {
      auto spt_ok = [](int v) { return v == 0 || v == 1 || v == 2 || v == 4 || v == 8; };
      if ((batch_block != 64 && batch_block != 128 && batch_block != 192 && batch_block != 256) ||
          (batch_spt != 1 && batch_spt != 2 && batch_spt != 4 && batch_spt != 8) || batch_grid < 0 || batch_grid > 64 ||
          batch_fuse < 0 || batch_fuse > 8 || !spt_ok(spt_mid) || !spt_ok(spt_wide)) {
        std::fclose(f);
        return fail(QD_EINVAL, "batch tuning entry out of range");
      }
      ++n;
    }
  }
  std::fclose(f);
  if (n == 0) return fail(QD_EINVAL, "no tuning entries in file");
  std::memcpy(g_table, tab, sizeof(tab));
  g_table_valid = true;
  if (batch_block) {
    TuneParams& tp = tune();
    tp.batch_block = batch_block;
    tp.batch_spt = batch_spt;
    if (batch_grid) tp.batch_wpc = batch_grid;
    if (batch_fuse) tp.batch_fuse = batch_fuse;
    tp.batch_spt_mid = spt_mid;
    tp.batch_spt_wide = spt_wide;
  }
  for (int k = 0; k < QD_BATCH_KEYS; ++k) tune().batch_spt_key[k] = key_spt[k];
  return QD_OK;
}

int qd_tune_save(const char* path) {
  if (!path) return fail(QD_EINVAL, "null path");
  return write_table(path);
}

}  // extern "C"
