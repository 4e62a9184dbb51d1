// Internal declarations shared by the host runtime and the kernel launchers of libqd.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "qd.h"
#include "qd_magic.h"

namespace qd {

// ------------------------------------------------------------------------------------------ limits
constexpr int kMaxGroups = 12;      // free-qudit groups a fast-path descriptor carries
constexpr int kMaxInlineDense = 9;  // dense U travels inside the kernel arguments up to d_T = 9
constexpr int kMaxInlineTable = 64; // diagonal / monomial tables inline up to d_T = 64
constexpr int kMaxTileRuns = 16;    // runs per LDS tile (product of the high targets' dims)
constexpr int kMaxTileCtl = 2;      // controls inside an LDS tile's suffix that the tile leaves out

// ------------------------------------------------------------------------------------------ errors
int fail(int code, const std::string& msg);   // records msg for qd_last_error, returns code
int hip_fail(hipError_t e, const char* what); // QD_EDEVICE / QD_ENOMEM with the HIP message

#define QD_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return ::qd::hip_fail(e_, #call); \
  } while (0)

// ------------------------------------------------------------------------------------------ register
struct Register {
  int n = 0;
  int32_t dims[QD_MAX_QUDITS] = {};
  int64_t strides[QD_MAX_QUDITS] = {};
  int64_t D = 0;
};

// Fills r from dims; returns QD_OK or an error code (validation of n, radices, overflow).
int make_register(const int32_t* dims, int32_t n, Register* r);

inline size_t amp_bytes(int prec) { return prec == QD_C128 ? 16 : 8; }

// ------------------------------------------------------------------------------------------ tuning
struct TuneParams {
  int direct_block = 256;   // threads per workgroup, slice-per-thread kernels
  int direct_spt = 2;       // slices per thread
  int tile_block = 256;     // threads per workgroup, LDS-tiled kernels
  int tile_elems = 2048;    // amplitudes per LDS tile (complex128; doubled for complex64)
  int diag_block = 256;
  int batch_block = 256;
  int batch_spt = 4;
  int batch_wpc = 64;       // batched layer kernel: 1..63 persistent workgroups per CU, 64 one per tile
  int batch_fuse = 1;       // gates composed into one batched operation (qd_batch_apply_layers, width 0)
  int batch_spt_mid = 0;    // slices per thread of batched slices of 5..9 amplitudes (0: two load batches)
  int batch_spt_wide = 0;   // slices per thread of batched slices of 12 to 32 amplitudes (0: as above)
  // batched slices per thread by (gate class, slice class, stride class), 0: the value above
  int batch_spt_key[QD_BATCH_KEYS] = {};
  int fused_cols = 64;      // slice columns per fused-block tile
  int run_min = 16;         // a target stride below this routes the gate to the LDS tile kernel
};
TuneParams& tune();
// key of a batched operation: composed (2+ gates) or one gate, slice size d_T, smallest target stride
int batch_key(bool composed, int dT, int64_t min_stride);

// Autotuned tile shape per (precision, stride class of the gate's smallest target stride).
constexpr int kStrideBuckets = 6;   // strides 1 | 2-3 | 4-15 | 16-255 | 256-4095 | >= 4096
struct TuneEntry {
  int valid;
  int tiled;        // stage slices in LDS
  int block;        // threads per workgroup
  int spt;          // slices per thread (direct kernel)
  int tile_elems;   // LDS tile budget in complex128 amplitudes (doubled for complex64)
};
int stride_bucket(int64_t s);
TuneEntry entry_for(int prec, int64_t min_stride);   // tuned entry, else the defaults above
void clear_tuned_table();

// ------------------------------------------------------------------------------------------ descriptors
// Linear work index -> element offset: base + sum_g digit_g(idx) * stride_g, digits taken in
// mixed radix over the groups, group 0 least significant. lmul gives each digit's weight in a
// second linear index (the local index of a diagonal's targets); zero for other groups.
struct SliceMap {
  uint32_t ng;
  uint32_t count;
  int64_t base;
  uint32_t gdim[kMaxGroups];
  uint32_t lmul[kMaxGroups];
  Magic32 gmag[kMaxGroups];
  int64_t gstride[kMaxGroups];
};

// 64-bit variant for the generic path (any register size); lives in device memory.
struct SliceMap64 {
  uint32_t ng;
  uint32_t pad;
  uint64_t count;
  int64_t base;
  uint64_t gdim[QD_MAX_QUDITS + 1];
  int64_t gstride[QD_MAX_QUDITS + 1];
};

struct Group {
  uint64_t dim;
  int64_t stride;
  uint32_t lmul;
};

// ------------------------------------------------------------------------------------------ state
struct ParamRing {            // pinned host staging + device copy for per-call parameters
  char* host = nullptr;
  char* dev = nullptr;
  size_t cap = 0;
  size_t head = 0;
};

}  // namespace qd

struct qd_state {
  qd::Register reg;
  int prec = QD_C128;
  void* data = nullptr;
  int64_t cap_bytes = 0;      // bytes of device memory at data (the library pads its own by 16)
  bool owned = false;
  hipStream_t stream = nullptr;
  int device = 0;
  qd::ParamRing ring;
  double* red = nullptr;      // reduction partials
  size_t red_cap = 0;         // in doubles
  void* mws = nullptr;        // measurement workspace (sums of weights, marginal partials, staging)
  size_t mws_cap = 0;         // in bytes
  int dens_n = 0;             // density matrix over dens_n qudits (register = dims ++ dims), else 0
  int64_t launches = 0;       // gate kernel launches made on the state (passes, for a density matrix)
};

namespace qd {

// Reserve `bytes` in the state's parameter ring, copy `src` there and return the device address.
// Wrapping around synchronises the stream first so no in-flight copy reads recycled memory.
int ring_push(qd_state* s, const void* src, size_t bytes, void** dev_out);
int ring_push_stream(ParamRing* r, hipStream_t stream, const void* src, size_t bytes, void** dev_out);
void ring_free(ParamRing* r);

// ------------------------------------------------------------------------------------------ gates
struct GatePlan {
  int cls = QD_CLASS_DENSE;
  int k = 0, m = 0;
  int32_t targets[QD_MAX_QUDITS];
  int32_t controls[QD_MAX_QUDITS];
  int32_t cvals[QD_MAX_QUDITS];
  int dT = 0;
  std::vector<double> U;        // 2 dT^2, dense
  std::vector<int32_t> dst;     // monomial: destination row of each column
  std::vector<double> ph;       // monomial: entry of column y (2 dT); diagonal: 2 dT phases
};

int validate_gate(const Register& r, const int32_t* targets, int32_t k, const int32_t* controls,
                  const int32_t* cvals, int32_t m, const double* U, uint32_t flags);
int classify(const double* U, int dT);
void make_plan(const Register& r, const int32_t* targets, int32_t k, const int32_t* controls,
               const int32_t* cvals, int32_t m, const double* U, GatePlan* p);
// make_plan, with controls of stride below one 128-byte line folded into the targets when the
// folded gate keeps a fast kernel (what qd_apply_gate launches)
void plan_gate(const Register& r, int prec, const int32_t* targets, int32_t k, const int32_t* controls,
               const int32_t* cvals, int32_t m, const double* U, GatePlan* p);

struct TileGeom {
  int pq = 0;          // first qudit of the low suffix staged in LDS
  uint64_t BL = 0;     // run length (amplitudes staged per run)
  uint64_t dH = 0;     // number of runs
  int nsc = 0;         // controls inside the suffix left out of the tile ...
  int sc[kMaxTileCtl] = {};  // ... their qudits, by increasing stride
};
bool tile_geometry(const Register& r, const GatePlan& p, int prec, TileGeom* g);
int route_gate(const Register& r, int prec, const GatePlan& p);

// Sparse state (qd_sparse.hip): its register, and a gate sequence applied with one parameter
// upload per run of monomial gates (all gates validated first; flags as qd_apply_gate_ex)
const Register& sparse_register(const qd_sparse* s);
struct SparseGate {
  std::vector<int32_t> t, c, v;   // targets, controls, control values
  std::vector<double> U;          // d_T x d_T, row-major, interleaved
};
int sparse_apply_gates(qd_sparse* s, const SparseGate* gates, size_t count, uint32_t flags);

// Launchers (qd_gates.hip)
int launch_gate(qd_state* s, const GatePlan& p);
const char* last_kernel();   // kernel instance of the calling thread's last gate or fused-block launch
void set_last_kernel(const char* name);   // (static storage; "" for none)
int launch_fill_basis(qd_state* s, int64_t index);
int launch_stream_copy(void* dst, const void* src, int64_t bytes, hipStream_t st);

// Readout (qd_reduce.hip)
int launch_probabilities(const qd_state* s, double* out_dev);
int reduce_norm2(const qd_state* s, double* out);
int reduce_probabilities_norm2(const qd_state* s, double* out_dev, double* norm2);   // one pass for both
int reduce_norm2_noalloc(const qd_state* s, double* out_dev);   // partials in a static device array
int reduce_compare(const qd_state* ref, const qd_state* s, double* max_abs, double* fid, double* drift,
                   double* norm2 = nullptr, double* fid_norm = nullptr);
int scale_state(qd_state* s, double f);
int normalize_on_device(qd_state* s);   // FP64 norm and scaling on the stream, no host wait

// Free-group construction: role[i] = 0 free, 1 fixed (excluded), 2 singleton (own group with
// lmul); qudits with index < lo or >= hi are ignored (treated as excluded).
std::vector<Group> make_groups(const Register& r, const int* role, const uint32_t* lmul, int lo, int hi);
int fill_slicemap(const std::vector<Group>& g, int64_t base, SliceMap* sm);
void fill_slicemap64(const std::vector<Group>& g, int64_t base, SliceMap64* sm);

}  // namespace qd
