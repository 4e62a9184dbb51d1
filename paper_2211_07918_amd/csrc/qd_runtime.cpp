// Host runtime of libqd: errors, registers, validation, named gates, gate classification and the
// state-vector API. No kernels here; launches go through the launchers in the .hip files.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "qd_internal.h"

namespace qd {

static thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(e == hipErrorOutOfMemory ? QD_ENOMEM : QD_EDEVICE, m);
}

TuneParams& tune() {
  static TuneParams t;
  return t;
}

int batch_key(bool composed, int dT, int64_t min_stride) {
  const int c = dT <= 4 ? 0 : (dT <= 9 ? 1 : 2);
  return 6 * (composed ? 1 : 0) + 2 * c + (min_stride < 16 ? 0 : 1);
}

// ------------------------------------------------------------------------------------------ register
int make_register(const int32_t* dims, int32_t n, Register* r) {
  if (!dims || !r) return fail(QD_EINVAL, "null dims");
  if (n < 1 || n > QD_MAX_QUDITS) return fail(QD_EINVAL, "number of qudits must be 1..64");
  r->n = n;
  int64_t D = 1;
  for (int i = n - 1; i >= 0; --i) {
    const int32_t d = dims[i];
    if (d < 2 || d > QD_MAX_RADIX) return fail(QD_EDIM, "qudit dimension must be 2..256");
    r->dims[i] = d;
    r->strides[i] = D;
    if (D > INT64_MAX / d) return fail(QD_EOVERFLOW, "register size overflows int64");
    D *= d;
  }
  r->D = D;
  return QD_OK;
}

// ------------------------------------------------------------------------------------------ named gates
// omega^m, omega = exp(2 pi i / d), exponent reduced mod d first, exact quarter turns.
static void omega_power(int64_t m, int d, double* re, double* im) {
  m %= d;
  if (m < 0) m += d;
  if ((4 * m) % d == 0) {
    static const double qr[4] = {1.0, 0.0, -1.0, 0.0};
    static const double qi[4] = {0.0, 1.0, 0.0, -1.0};
    const int q = int((4 * m) / d);
    *re = qr[q];
    *im = qi[q];
    return;
  }
  const double ang = 2.0 * M_PI * double(m) / double(d);
  *re = std::cos(ang);
  *im = std::sin(ang);
}

}  // namespace qd

using namespace qd;

extern "C" {

const char* qd_version(void) { return "libqd 1.0 (gfx950)"; }

const char* qd_last_error(void) { return g_last_error.c_str(); }

const char* qd_last_kernel(void) { return last_kernel(); }

int qd_register_strides(const int32_t* dims, int32_t n, int64_t* D_out, int64_t* strides_out) {
  if (!D_out || !strides_out) return fail(QD_EINVAL, "null output");
  Register r;
  int rc = make_register(dims, n, &r);
  if (rc) return rc;
  *D_out = r.D;
  for (int i = 0; i < n; ++i) strides_out[i] = r.strides[i];
  return QD_OK;
}

int qd_gate_matrix(int32_t kind, int32_t d, int32_t a, double* U) {
  if (!U) return fail(QD_EINVAL, "null output");
  if (d < 2 || d > QD_MAX_RADIX) return fail(QD_EDIM, "dimension must be 2..256");
  std::memset(U, 0, sizeof(double) * 2 * d * d);
  auto at = [&](int r, int c) { return U + 2 * (size_t(r) * d + c); };
  switch (kind) {
    case QD_GATE_X:  // |x> -> |(x + a) mod d>, 1 <= a <= d - 1 (Sec. 2.1, generalized NOT)
      if (a < 1 || a > d - 1) return fail(QD_EINVAL, "shift must satisfy 1 <= a <= d-1");
      for (int x = 0; x < d; ++x) at((x + a) % d, x)[0] = 1.0;
      return QD_OK;
    case QD_GATE_Z:  // diag(omega^x) (Sec. 2.1, generalized phase-shift)
      for (int x = 0; x < d; ++x) omega_power(x, d, at(x, x), at(x, x) + 1);
      return QD_OK;
    case QD_GATE_F: {  // (1/sqrt d) omega^{jk} (Sec. 2.1, generalized Hadamard)
      const double s = 1.0 / std::sqrt(double(d));
      for (int j = 0; j < d; ++j)
        for (int k = 0; k < d; ++k) {
          double re, im;
          omega_power(int64_t(j) * k, d, &re, &im);
          at(j, k)[0] = re * s;
          at(j, k)[1] = im * s;
        }
      return QD_OK;
    }
    case QD_GATE_I:
      for (int x = 0; x < d; ++x) at(x, x)[0] = 1.0;
      return QD_OK;
    default:
      return fail(QD_EINVAL, "unknown gate kind");
  }
}

}  // extern "C"

namespace qd {

// ------------------------------------------------------------------------------------------ validation
int validate_gate(const Register& r, const int32_t* targets, int32_t k, const int32_t* controls,
                  const int32_t* cvals, int32_t m, const double* U, uint32_t flags) {
  if (!targets || k < 1) return fail(QD_EINVAL, "a gate needs at least one target");
  if (m < 0 || (m > 0 && (!controls || !cvals))) return fail(QD_EINVAL, "bad control arrays");
  if (k + m > r.n) return fail(QD_EINVAL, "more targets and controls than qudits");
  if (!U) return fail(QD_EINVAL, "null U");
  bool used[QD_MAX_QUDITS] = {};
  int64_t dT = 1;
  for (int j = 0; j < k; ++j) {
    const int t = targets[j];
    if (t < 0 || t >= r.n) return fail(QD_EINVAL, "target out of range");
    if (used[t]) return fail(QD_EINVAL, "duplicate target");
    used[t] = true;
    dT *= r.dims[t];
    if (dT > QD_MAX_GATE_DIM) return fail(QD_EDIM, "gate dimension d_T exceeds 1024");
  }
  for (int j = 0; j < m; ++j) {
    const int c = controls[j];
    if (c < 0 || c >= r.n) return fail(QD_EINVAL, "control out of range");
    if (used[c]) return fail(QD_EINVAL, "control repeats a target or a control");
    used[c] = true;
    if (cvals[j] < 0 || cvals[j] >= r.dims[c]) return fail(QD_EINVAL, "control value outside 0..d_c-1");
  }
  const size_t nn = size_t(dT) * size_t(dT);
  for (size_t i = 0; i < 2 * nn; ++i)
    if (!std::isfinite(U[i])) return fail(QD_ENOTUNITARY, "U has a NaN or Inf entry");
  if (flags & QD_FLAG_SKIP_UNITARY_CHECK) return QD_OK;
  // max_{ij} |(U^dag U)_{ij} - delta_ij| <= 1e-10 in FP64
  const int n = int(dT);
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) {
      double re = 0.0, im = 0.0;
      for (int l = 0; l < n; ++l) {
        const double ar = U[2 * (size_t(l) * n + i)], ai = -U[2 * (size_t(l) * n + i) + 1];
        const double br = U[2 * (size_t(l) * n + j)], bi = U[2 * (size_t(l) * n + j) + 1];
        re += ar * br - ai * bi;
        im += ar * bi + ai * br;
      }
      if (i == j) re -= 1.0;
      if (std::sqrt(re * re + im * im) > 1e-10) return fail(QD_ENOTUNITARY, "U is not unitary within 1e-10");
    }
  return QD_OK;
}

int classify(const double* U, int dT) {
  auto nz = [&](int r, int c) {
    const double* e = U + 2 * (size_t(r) * dT + c);
    return e[0] != 0.0 || e[1] != 0.0;
  };
  bool diag = true;
  for (int r = 0; r < dT && diag; ++r)
    for (int c = 0; c < dT; ++c)
      if (r != c && nz(r, c)) { diag = false; break; }
  if (diag) return QD_CLASS_DIAGONAL;
  std::vector<int> rowcount(dT, 0);
  for (int c = 0; c < dT; ++c) {
    int cnt = 0;
    for (int r = 0; r < dT; ++r)
      if (nz(r, c)) { ++cnt; ++rowcount[r]; }
    if (cnt != 1) return QD_CLASS_DENSE;
  }
  for (int r = 0; r < dT; ++r)
    if (rowcount[r] != 1) return QD_CLASS_DENSE;
  return QD_CLASS_MONOMIAL;
}

void make_plan(const Register& r, const int32_t* targets, int32_t k, const int32_t* controls,
               const int32_t* cvals, int32_t m, const double* U, GatePlan* p) {
  p->k = k;
  p->m = m;
  int dT = 1;
  for (int j = 0; j < k; ++j) {
    p->targets[j] = targets[j];
    dT *= r.dims[targets[j]];
  }
  for (int j = 0; j < m; ++j) {
    p->controls[j] = controls[j];
    p->cvals[j] = cvals[j];
  }
  p->dT = dT;
  p->cls = classify(U, dT);
  p->U.assign(U, U + 2 * size_t(dT) * dT);
  p->dst.clear();
  p->ph.clear();
  if (p->cls == QD_CLASS_DIAGONAL) {
    p->ph.resize(2 * dT);
    for (int y = 0; y < dT; ++y) {
      p->ph[2 * y] = U[2 * (size_t(y) * dT + y)];
      p->ph[2 * y + 1] = U[2 * (size_t(y) * dT + y) + 1];
    }
  } else if (p->cls == QD_CLASS_MONOMIAL) {
    p->dst.resize(dT);
    p->ph.resize(2 * dT);
    for (int c = 0; c < dT; ++c)
      for (int rr = 0; rr < dT; ++rr) {
        const double* e = U + 2 * (size_t(rr) * dT + c);
        if (e[0] != 0.0 || e[1] != 0.0) {
          p->dst[c] = rr;
          p->ph[2 * c] = e[0];
          p->ph[2 * c + 1] = e[1];
        }
      }
  }
}

// A control whose stride is below one 128-byte line of amplitudes leaves every line partly
// active: a pass over the matching slices still moves whole lines, and with its partial writes
// such gates measured slower than a full pass (about 1 ms against 0.57 ms on a 1.7 GB state).
// Where no kernel writes those lines whole for the gate as given (diagonal gates, dense d_T above
// 9), such controls become targets of an embedded gate (U where they hold their values, the
// identity elsewhere, exactly), which one coalesced pass applies, provided it keeps a fast kernel.
void plan_gate(const Register& r, int prec, const int32_t* targets, int32_t k, const int32_t* controls,
               const int32_t* cvals, int32_t m, const double* U, GatePlan* p) {
  make_plan(r, targets, k, controls, cvals, m, U, p);
  const int64_t line = prec == QD_C128 ? 8 : 16;
  std::vector<int> low, keep;
  for (int j = 0; j < m; ++j) (r.strides[controls[j]] < line ? low : keep).push_back(j);
  if (low.empty()) return;
  // The slice-per-thread kernel takes such controls as free digits tested per slice, and the LDS
  // tile kernel stages every value of a control inside its suffix and mixes the matching slices
  // only: both write whole lines while mixing d_T amplitudes per slice, so no folding there.
  const int route0 = route_gate(r, prec, *p);
  if (route0 == QD_ROUTE_TILED) return;
  if (route0 == QD_ROUTE_DIRECT && (p->cls == QD_CLASS_MONOMIAL || p->dT <= kMaxInlineDense)) return;
  int dC = 1;
  for (int j : low) dC *= r.dims[controls[j]];
  const int dT = p->dT, dG = dT * dC;
  if (dG > QD_MAX_GATE_DIM) return;
  int vidx = 0;                         // local index of the absorbed controls' values
  for (int j : low) vidx = vidx * r.dims[controls[j]] + cvals[j];
  std::vector<double> G(2 * size_t(dG) * dG, 0.0);
  for (int c = 0; c < dC; ++c)
    for (int t = 0; t < dT; ++t)
      for (int t1 = 0; t1 < dT; ++t1) {
        const size_t o = 2 * (size_t(t * dC + c) * dG + size_t(t1 * dC + c));
        if (c == vidx) {
          G[o] = U[2 * (size_t(t) * dT + t1)];
          G[o + 1] = U[2 * (size_t(t) * dT + t1) + 1];
        } else if (t == t1) {
          G[o] = 1.0;
        }
      }
  std::vector<int32_t> t2(targets, targets + k), c2, v2;
  for (int j : low) t2.push_back(controls[j]);
  for (int j : keep) {
    c2.push_back(controls[j]);
    v2.push_back(cvals[j]);
  }
  GatePlan q;
  make_plan(r, t2.data(), int32_t(t2.size()), c2.data(), v2.data(), int32_t(c2.size()), G.data(), &q);
  const int route = route_gate(r, prec, q);   // fold only into the slice-per-thread, tiled or diagonal kernels
  if (route != QD_ROUTE_GENERIC && route != QD_ROUTE_GEMM) *p = std::move(q);
}

// ------------------------------------------------------------------------------------------ groups
std::vector<Group> make_groups(const Register& r, const int* role, const uint32_t* lmul, int lo, int hi) {
  std::vector<Group> g;
  uint64_t run = 1;
  int64_t run_stride = 0;
  auto close = [&]() {
    if (run > 1) g.push_back(Group{run, run_stride, 0});
    run = 1;
  };
  for (int i = r.n - 1; i >= 0; --i) {
    const bool inside = i >= lo && i < hi;
    const int ro = inside ? role[i] : 1;
    if (ro == 0) {
      if (run == 1) run_stride = r.strides[i];
      run *= uint64_t(r.dims[i]);
    } else {
      close();
      if (ro == 2) g.push_back(Group{uint64_t(r.dims[i]), r.strides[i], lmul ? lmul[i] : 0});
    }
  }
  close();
  return g;
}

int fill_slicemap(const std::vector<Group>& g, int64_t base, SliceMap* sm) {
  std::memset(sm, 0, sizeof(*sm));
  if (int(g.size()) > kMaxGroups) return fail(QD_EINVAL, "too many index groups for the fast path");
  uint64_t count = 1;
  for (size_t i = 0; i < g.size(); ++i) {
    count *= g[i].dim;
    sm->gdim[i] = uint32_t(g[i].dim);
    sm->gstride[i] = g[i].stride;
    sm->lmul[i] = g[i].lmul;
    sm->gmag[i] = make_magic32(uint32_t(g[i].dim));
  }
  if (count > 0xFFFFFFFFull) return fail(QD_EOVERFLOW, "work count exceeds 32 bits");
  sm->ng = uint32_t(g.size());
  sm->count = uint32_t(count);
  sm->base = base;
  return QD_OK;
}

void fill_slicemap64(const std::vector<Group>& g, int64_t base, SliceMap64* sm) {
  std::memset(sm, 0, sizeof(*sm));
  uint64_t count = 1;
  for (size_t i = 0; i < g.size(); ++i) {
    count *= g[i].dim;
    sm->gdim[i] = g[i].dim;
    sm->gstride[i] = g[i].stride;
  }
  sm->ng = uint32_t(g.size());
  sm->count = count;
  sm->base = base;
}

// ------------------------------------------------------------------------------------------ param ring
int ring_push_stream(ParamRing* r, hipStream_t stream, const void* src, size_t bytes, void** dev_out) {
  const size_t align = 256;
  const size_t need = (bytes + align - 1) / align * align;
  if (!r->host || need > r->cap) {
    if (r->host) {
      // earlier copies and the kernels reading them must finish before the buffers go away
      QD_HIP(hipStreamSynchronize(stream));
      ring_free(r);
    }
    r->cap = size_t(8) << 20;
    while (r->cap < need) r->cap *= 2;
    QD_HIP(hipHostMalloc((void**)&r->host, r->cap, hipHostMallocDefault));
    QD_HIP(hipMalloc((void**)&r->dev, r->cap));
    r->head = 0;
  }
  if (r->head + need > r->cap) {
    // every earlier copy out of the ring must have finished before the host rewrites it
    QD_HIP(hipStreamSynchronize(stream));
    r->head = 0;
  }
  std::memcpy(r->host + r->head, src, bytes);
  QD_HIP(hipMemcpyAsync(r->dev + r->head, r->host + r->head, bytes, hipMemcpyHostToDevice, stream));
  *dev_out = r->dev + r->head;
  r->head += need;
  return QD_OK;
}

int ring_push(qd_state* s, const void* src, size_t bytes, void** dev_out) {
  return ring_push_stream(&s->ring, s->stream, src, bytes, dev_out);
}

void ring_free(ParamRing* r) {
  if (r->host) (void)hipHostFree(r->host);
  if (r->dev) (void)hipFree(r->dev);
  r->host = r->dev = nullptr;
  r->cap = r->head = 0;
}

}  // namespace qd

// ------------------------------------------------------------------------------------------ state API
extern "C" {

int qd_validate_gate(const int32_t* dims, int32_t n, const int32_t* targets, int32_t k,
                     const int32_t* controls, const int32_t* control_values, int32_t m,
                     const double* U, uint32_t flags) {
  Register r;
  int rc = make_register(dims, n, &r);
  if (rc) return rc;
  return validate_gate(r, targets, k, controls, control_values, m, U, flags);
}

int qd_gate_route(const int32_t* dims, int32_t n, int32_t prec, const int32_t* targets, int32_t k,
                  const int32_t* controls, const int32_t* control_values, int32_t m, const double* U,
                  int32_t* route_out) {
  if (!route_out) return fail(QD_EINVAL, "null output");
  if (prec != QD_C128 && prec != QD_C64) return fail(QD_EINVAL, "precision must be QD_C128 or QD_C64");
  Register r;
  int rc = make_register(dims, n, &r);
  if (rc) return rc;
  rc = validate_gate(r, targets, k, controls, control_values, m, U, QD_FLAG_SKIP_UNITARY_CHECK);
  if (rc) return rc;
  GatePlan p;
  plan_gate(r, prec, targets, k, controls, control_values, m, U, &p);
  *route_out = route_gate(r, prec, p);
  return QD_OK;
}

int qd_gate_class(const double* U, int32_t dT) {
  if (!U || dT < 1 || dT > QD_MAX_GATE_DIM) return -1;
  return classify(U, dT);
}

static int new_state(const int32_t* dims, int32_t n, int32_t prec, void* stream, qd_state** out) {
  if (!out) return fail(QD_EINVAL, "null output handle");
  if (prec != QD_C128 && prec != QD_C64) return fail(QD_EINVAL, "precision must be QD_C128 or QD_C64");
  auto* s = new qd_state();
  int rc = make_register(dims, n, &s->reg);
  if (rc) {
    delete s;
    return rc;
  }
  if (s->reg.D > INT64_MAX / int64_t(amp_bytes(prec))) {
    delete s;
    return fail(QD_EOVERFLOW, "state size in bytes overflows int64");
  }
  s->prec = prec;
  s->stream = (hipStream_t)stream;
  (void)hipGetDevice(&s->device);
  *out = s;
  return QD_OK;
}

int qd_state_init(const int32_t* dims, int32_t n, int32_t prec, void* hip_stream, qd_state** out) {
  qd_state* s = nullptr;
  int rc = new_state(dims, n, prec, hip_stream, &s);
  if (rc) return rc;
  // 16 spare bytes: a kernel may read one 16-byte unit that ends past the last amplitude (and never
  // writes it)
  const size_t bytes = size_t(s->reg.D) * amp_bytes(prec) + 16;
  hipError_t e = hipMalloc(&s->data, bytes);
  if (e != hipSuccess) {
    delete s;
    (void)hipGetLastError();
    return fail(QD_ENOMEM, "device allocation of the state failed (" + std::to_string(bytes) + " bytes)");
  }
  s->cap_bytes = int64_t(bytes);
  s->owned = true;
  rc = launch_fill_basis(s, 0);
  if (rc) {
    qd_state_free(s);
    return rc;
  }
  *out = s;
  return QD_OK;
}

int qd_state_wrap(const int32_t* dims, int32_t n, int32_t prec, void* dev_ptr, int64_t bytes,
                  void* hip_stream, qd_state** out) {
  if (!dev_ptr) return fail(QD_EINVAL, "null device pointer");
  qd_state* s = nullptr;
  int rc = new_state(dims, n, prec, hip_stream, &s);
  if (rc) return rc;
  if (bytes < 0 || uint64_t(bytes) < uint64_t(s->reg.D) * amp_bytes(prec)) {
    delete s;
    return fail(QD_EDIM, "wrapped buffer is smaller than the state");
  }
  s->data = dev_ptr;
  s->cap_bytes = bytes;
  s->owned = false;
  *out = s;
  return QD_OK;
}

int qd_state_set_basis(qd_state* s, const int32_t* values) {
  if (!s || !values) return fail(QD_EINVAL, "null argument");
  int64_t idx = 0;
  for (int i = 0; i < s->reg.n; ++i) {
    if (values[i] < 0 || values[i] >= s->reg.dims[i]) return fail(QD_EINVAL, "basis value outside 0..d-1");
    idx += int64_t(values[i]) * s->reg.strides[i];
  }
  return launch_fill_basis(s, idx);
}

int qd_state_upload(qd_state* s, const void* host, int64_t n) {
  if (!s || !host) return fail(QD_EINVAL, "null argument");
  if (n != s->reg.D) return fail(QD_EDIM, "amplitude count differs from D");
  QD_HIP(hipMemcpyAsync(s->data, host, size_t(n) * amp_bytes(s->prec), hipMemcpyHostToDevice, s->stream));
  QD_HIP(hipStreamSynchronize(s->stream));
  return QD_OK;
}

int qd_state_download(const qd_state* s, void* host, int64_t n) {
  if (!s || !host) return fail(QD_EINVAL, "null argument");
  if (n != s->reg.D) return fail(QD_EDIM, "amplitude count differs from D");
  QD_HIP(hipMemcpyAsync(host, s->data, size_t(n) * amp_bytes(s->prec), hipMemcpyDeviceToHost, s->stream));
  QD_HIP(hipStreamSynchronize(s->stream));
  return QD_OK;
}

int qd_state_size(const qd_state* s, int64_t* D) {
  if (!s || !D) return fail(QD_EINVAL, "null argument");
  *D = s->reg.D;
  return QD_OK;
}

int qd_state_dims(const qd_state* s, int32_t* dims, int32_t* n) {
  if (!s || !dims || !n) return fail(QD_EINVAL, "null argument");
  for (int i = 0; i < s->reg.n; ++i) dims[i] = s->reg.dims[i];
  *n = s->reg.n;
  return QD_OK;
}

int qd_state_precision(const qd_state* s, int32_t* p) {
  if (!s || !p) return fail(QD_EINVAL, "null argument");
  *p = s->prec;
  return QD_OK;
}

int qd_state_device_ptr(const qd_state* s, void** p) {
  if (!s || !p) return fail(QD_EINVAL, "null argument");
  *p = s->data;
  return QD_OK;
}

int qd_state_sync(const qd_state* s) {
  if (!s) return fail(QD_EINVAL, "null state");
  QD_HIP(hipStreamSynchronize(s->stream));
  QD_HIP(hipGetLastError());
  return QD_OK;
}

void qd_state_free(qd_state* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  if (s->owned && s->data) (void)hipFree(s->data);
  if (s->red) (void)hipFree(s->red);
  if (s->mws) (void)hipFree(s->mws);
  ring_free(&s->ring);
  delete s;
}

int qd_apply_gate_ex(qd_state* s, const int32_t* targets, int32_t k, const int32_t* controls,
                     const int32_t* control_values, int32_t m, const double* U, uint32_t flags) {
  if (!s) return fail(QD_EINVAL, "null state");
  int rc = validate_gate(s->reg, targets, k, controls, control_values, m, U, flags);
  if (rc) return rc;
  GatePlan p;
  plan_gate(s->reg, s->prec, targets, k, controls, control_values, m, U, &p);
  rc = launch_gate(s, p);
  if (rc == QD_OK && last_kernel()[0]) ++s->launches;
  return rc;
}

int qd_state_gate_launches(const qd_state* s, int64_t* out) {
  if (!s || !out) return fail(QD_EINVAL, "null argument");
  *out = s->launches;
  return QD_OK;
}

int qd_apply_gate(qd_state* s, const int32_t* targets, int32_t k, const int32_t* controls,
                  const int32_t* control_values, int32_t m, const double* U) {
  return qd_apply_gate_ex(s, targets, k, controls, control_values, m, U, 0);
}

int qd_probabilities(const qd_state* s, double* out, int32_t out_is_device) {
  if (!s || !out) return fail(QD_EINVAL, "null argument");
  if (out_is_device) return launch_probabilities(s, out);
  double* dev = nullptr;
  const size_t bytes = size_t(s->reg.D) * sizeof(double);
  QD_HIP(hipMalloc((void**)&dev, bytes));
  int rc = launch_probabilities(s, dev);
  if (!rc) {
    hipError_t e = hipMemcpyAsync(out, dev, bytes, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) rc = hip_fail(e, "probabilities download");
  }
  (void)hipFree(dev);
  return rc;
}

int qd_probabilities_norm2(const qd_state* s, double* out, int32_t out_is_device, double* norm2) {
  if (!s || !out || !norm2) return fail(QD_EINVAL, "null argument");
  if (out_is_device) return reduce_probabilities_norm2(s, out, norm2);
  double* dev = nullptr;
  const size_t bytes = size_t(s->reg.D) * sizeof(double);
  QD_HIP(hipMalloc((void**)&dev, bytes));
  int rc = reduce_probabilities_norm2(s, dev, norm2);
  if (!rc) {
    hipError_t e = hipMemcpyAsync(out, dev, bytes, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) rc = hip_fail(e, "probabilities download");
  }
  (void)hipFree(dev);
  return rc;
}

int qd_norm2(const qd_state* s, double* out) {
  if (!s || !out) return fail(QD_EINVAL, "null argument");
  return reduce_norm2(s, out);
}

int qd_norm2_noalloc(const qd_state* s, double* out_dev) {
  if (!s || !out_dev) return fail(QD_EINVAL, "null argument");
  return reduce_norm2_noalloc(s, out_dev);
}

static int check_compare_args(const qd_state* ref, const qd_state* s) {
  if (!ref || !s) return fail(QD_EINVAL, "null state");
  if (ref->prec != QD_C128) return fail(QD_EDIM, "reference state must be complex128");
  if (ref->reg.n != s->reg.n || ref->reg.D != s->reg.D) return fail(QD_EDIM, "registers differ");
  for (int i = 0; i < s->reg.n; ++i)
    if (ref->reg.dims[i] != s->reg.dims[i]) return fail(QD_EDIM, "registers differ");
  return QD_OK;
}

int qd_compare(const qd_state* ref, const qd_state* s, double* max_abs, double* fid, double* drift) {
  int rc = check_compare_args(ref, s);
  if (rc) return rc;
  return reduce_compare(ref, s, max_abs, fid, drift);
}

int qd_compare_ex(const qd_state* ref, const qd_state* s, double* out) {
  if (!out) return fail(QD_EINVAL, "null output");
  int rc = check_compare_args(ref, s);
  if (rc) return rc;
  return reduce_compare(ref, s, &out[0], &out[1], &out[2], &out[3], &out[4]);
}

int qd_normalize(qd_state* s, double* before) {
  if (!s) return fail(QD_EINVAL, "null state");
  double n2 = 0.0;
  int rc = reduce_norm2(s, &n2);
  if (rc) return rc;
  if (before) *before = n2;
  if (!(n2 > 0.0) || !std::isfinite(n2)) return fail(QD_EINVAL, "state norm is zero or not finite");
  return scale_state(s, 1.0 / std::sqrt(n2));
}

int qd_stream_copy(void* dst, const void* src, int64_t bytes, void* hip_stream) {
  if (!dst || !src || bytes < 0) return fail(QD_EINVAL, "bad copy arguments");
  if (bytes % 16) return fail(QD_EINVAL, "copy size must be a multiple of 16 bytes");
  return launch_stream_copy(dst, src, bytes, (hipStream_t)hip_stream);
}

int qd_tune_set(int32_t param, int32_t value) {
  clear_tuned_table();  // explicit settings replace an autotuned table
  TuneParams& t = tune();
  const TuneParams def;
  auto blk = [&](int v, int d) { return v == 0 ? d : v; };
  if (value < 0) return fail(QD_EINVAL, "negative tuning value");
  switch (param) {
    case QD_TUNE_DIRECT_BLOCK:
    case QD_TUNE_TILE_BLOCK:
    case QD_TUNE_DIAG_BLOCK:
    case QD_TUNE_BATCH_BLOCK:
      if (value != 0 && (value % 64 || value > 256)) return fail(QD_EINVAL, "block must be 64, 128, 192 or 256");
      if (param == QD_TUNE_DIRECT_BLOCK) t.direct_block = blk(value, def.direct_block);
      if (param == QD_TUNE_TILE_BLOCK) t.tile_block = blk(value, def.tile_block);
      if (param == QD_TUNE_DIAG_BLOCK) t.diag_block = blk(value, def.diag_block);
      if (param == QD_TUNE_BATCH_BLOCK) t.batch_block = blk(value, def.batch_block);
      return QD_OK;
    case QD_TUNE_DIRECT_SPT:
      if (value != 0 && value != 1 && value != 2 && value != 4) return fail(QD_EINVAL, "slices per thread must be 1, 2 or 4");
      t.direct_spt = blk(value, def.direct_spt);
      return QD_OK;
    case QD_TUNE_BATCH_SPT:
      if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8)
        return fail(QD_EINVAL, "batch slices per thread must be 1, 2, 4 or 8");
      t.batch_spt = blk(value, def.batch_spt);
      return QD_OK;
    case QD_TUNE_TILE_ELEMS:
      if (value != 0 && (value < 256 || value > 4096 || (value & (value - 1)))) return fail(QD_EINVAL, "tile must be a power of two in 256..4096");
      t.tile_elems = blk(value, def.tile_elems);
      return QD_OK;
    case QD_TUNE_FUSED_COLS:
      if (value != 0 && value != 32 && value != 64 && value != 128) return fail(QD_EINVAL, "fused columns must be 32, 64 or 128");
      t.fused_cols = blk(value, def.fused_cols);
      return QD_OK;
    case QD_TUNE_RUN_MIN:
      if (value > 1024) return fail(QD_EINVAL, "run threshold must be 1..1024");
      t.run_min = blk(value, def.run_min);
      return QD_OK;
    case QD_TUNE_BATCH_GRID:
      if (value > 64) return fail(QD_EINVAL, "workgroups per compute unit must be 1..64");
      t.batch_wpc = blk(value, def.batch_wpc);
      return QD_OK;
    case QD_TUNE_BATCH_FUSE:
      if (value > 8) return fail(QD_EINVAL, "fusion width must be 1..8");
      t.batch_fuse = blk(value, def.batch_fuse);
      return QD_OK;
    case QD_TUNE_BATCH_SPT_MID:
    case QD_TUNE_BATCH_SPT_WIDE:
      if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8)
        return fail(QD_EINVAL, "batch slices per thread must be 0 (the default rule), 1, 2, 4 or 8");
      (param == QD_TUNE_BATCH_SPT_MID ? t.batch_spt_mid : t.batch_spt_wide) = value;
      return QD_OK;
    default:
      return fail(QD_EINVAL, "unknown tuning parameter");
  }
}

int qd_batch_tune_key_set(int32_t key, int32_t spt) {
  if (key < 0 || key >= QD_BATCH_KEYS) return fail(QD_EINVAL, "batch tuning key must be 0..11");
  if (spt != 0 && spt != 1 && spt != 2 && spt != 4 && spt != 8)
    return fail(QD_EINVAL, "batch slices per thread must be 0 (inherit), 1, 2, 4 or 8");
  tune().batch_spt_key[key] = spt;
  return QD_OK;
}

int qd_batch_tune_key_get(int32_t key, int32_t* spt) {
  if (!spt) return fail(QD_EINVAL, "null output");
  if (key < 0 || key >= QD_BATCH_KEYS) return fail(QD_EINVAL, "batch tuning key must be 0..11");
  *spt = tune().batch_spt_key[key];
  return QD_OK;
}

int qd_tune_get(int32_t param, int32_t* value) {
  if (!value) return fail(QD_EINVAL, "null output");
  const TuneParams& t = tune();
  switch (param) {
    case QD_TUNE_DIRECT_BLOCK: *value = t.direct_block; return QD_OK;
    case QD_TUNE_DIRECT_SPT: *value = t.direct_spt; return QD_OK;
    case QD_TUNE_TILE_BLOCK: *value = t.tile_block; return QD_OK;
    case QD_TUNE_TILE_ELEMS: *value = t.tile_elems; return QD_OK;
    case QD_TUNE_DIAG_BLOCK: *value = t.diag_block; return QD_OK;
    case QD_TUNE_BATCH_BLOCK: *value = t.batch_block; return QD_OK;
    case QD_TUNE_BATCH_SPT: *value = t.batch_spt; return QD_OK;
    case QD_TUNE_FUSED_COLS: *value = t.fused_cols; return QD_OK;
    case QD_TUNE_RUN_MIN: *value = t.run_min; return QD_OK;
    case QD_TUNE_BATCH_GRID: *value = t.batch_wpc; return QD_OK;
    case QD_TUNE_BATCH_FUSE: *value = t.batch_fuse; return QD_OK;
    case QD_TUNE_BATCH_SPT_MID: *value = t.batch_spt_mid; return QD_OK;
    case QD_TUNE_BATCH_SPT_WIDE: *value = t.batch_spt_wide; return QD_OK;
    default: return fail(QD_EINVAL, "unknown tuning parameter");
  }
}

}  // extern "C"
