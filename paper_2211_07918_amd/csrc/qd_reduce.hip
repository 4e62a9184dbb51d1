// Readout kernels (Sec. 3.8): probabilities |alpha_x|^2 in FP64, the squared norm, and the
// precision diagnostics of a state against a complex128 reference. All sums are deterministic:
// a fixed grid (a function of D only) reduces fixed strided subsets in a fixed tree order, then a
// single workgroup reduces the partials in a fixed order, so reruns are bitwise identical.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "qd_internal.h"
#include "qd_stream.h"

namespace qd {

constexpr int kRedBlock = 256;
constexpr int kRedMaxGrid = 2048;

template <typename R> struct CxR;
template <> struct CxR<double> { using T = double2; };
template <> struct CxR<float> { using T = float2; };

static unsigned red_grid(uint64_t D) {
  return unsigned(std::max<uint64_t>(1, std::min<uint64_t>(kRedMaxGrid, (D + kRedBlock * 8 - 1) / (kRedBlock * 8))));
}

// |alpha|^2 in FP64, written as one fused multiply-add so that the probability pass, the norm pass
// and the fused pass below all round it the same way
template <typename C>
__device__ __forceinline__ double prob_of(const C a) {
  const double re = double(a.x), im = double(a.y);
  return fma(re, re, im * im);
}

// one amplitude per thread, streaming access (faster than a grid-stride loop on gfx950)
template <typename R>
__global__ __launch_bounds__(256) void k_probabilities(const R* psi_raw, double* __restrict__ p, uint64_t D) {
  using C = typename CxR<R>::T;
  const C* psi = reinterpret_cast<const C*>(psi_raw);
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < D) __builtin_nontemporal_store(prob_of(ld_stream(psi + i)), p + i);
}

// NV values per thread, reduced by sum (slot < NSUM) or max (other slots)
template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], int nsum, double* out) {
  __shared__ double sh[NV][kRedBlock];
#pragma unroll
  for (int q = 0; q < NV; ++q) sh[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int w = kRedBlock / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const double a = sh[q][threadIdx.x], b = sh[q][threadIdx.x + w];
        sh[q][threadIdx.x] = q < nsum ? a + b : fmax(a, b);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) out[q] = sh[q][0];
}

template <typename R>
__global__ __launch_bounds__(256) void k_norm_partial(const R* psi_raw, uint64_t D, double* partial) {
  using C = typename CxR<R>::T;
  const C* psi = reinterpret_cast<const C*>(psi_raw);
  double v[1] = {0.0};
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < D; i += uint64_t(gridDim.x) * blockDim.x)
    v[0] += prob_of(ld_stream(psi + i));
  block_reduce<1>(v, 1, partial + blockIdx.x);
}

// Probabilities and the norm's partial sums in one pass over the state: the grid, the amplitudes
// each thread visits, their order and the tree are those of k_norm_partial, so the partials (and
// the norm k_finish makes of them) are bitwise those of qd_norm2, and every probability is the value
// k_probabilities writes.
template <typename R>
__global__ __launch_bounds__(256) void k_probabilities_norm(const R* psi_raw, double* __restrict__ p, uint64_t D,
                                                            double* partial) {
  using C = typename CxR<R>::T;
  const C* psi = reinterpret_cast<const C*>(psi_raw);
  double v[1] = {0.0};
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < D; i += uint64_t(gridDim.x) * blockDim.x) {
    const double q = prob_of(ld_stream(psi + i));
    __builtin_nontemporal_store(q, p + i);
    v[0] += q;
  }
  block_reduce<1>(v, 1, partial + blockIdx.x);
}

// slots: 0 Re<ref|s>, 1 Im<ref|s>, 2 ||s||^2, 3 max |s - ref|
template <typename R>
__global__ __launch_bounds__(256) void k_compare_partial(const double* ref_raw, const R* s_raw, uint64_t D, double* partial) {
  using C = typename CxR<R>::T;
  const double2* ref = reinterpret_cast<const double2*>(ref_raw);
  const C* s = reinterpret_cast<const C*>(s_raw);
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < D; i += uint64_t(gridDim.x) * blockDim.x) {
    const double2 a = ld_stream(ref + i);
    const C b = ld_stream(s + i);
    const double br = double(b.x), bi = double(b.y);
    v[0] += a.x * br + a.y * bi;   // conj(a) * b
    v[1] += a.x * bi - a.y * br;
    v[2] += br * br + bi * bi;
    const double dr = br - a.x, di = bi - a.y;
    v[3] = fmax(v[3], sqrt(dr * dr + di * di));
  }
  double* out = partial + 4 * size_t(blockIdx.x);
  block_reduce<4>(v, 3, out);
}

template <int NV>
__global__ __launch_bounds__(256) void k_finish(const double* partial, unsigned n, int nsum, double* out) {
  double v[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = 0.0;
  for (unsigned i = threadIdx.x; i < n; i += blockDim.x)
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const double x = partial[size_t(i) * NV + q];
      v[q] = q < nsum ? v[q] + x : fmax(v[q], x);
    }
  block_reduce<NV>(v, nsum, out);
}

static int ensure_red(qd_state* s, size_t doubles) {
  if (s->red_cap >= doubles) return QD_OK;
  if (s->red) (void)hipFree(s->red);
  s->red = nullptr;
  s->red_cap = 0;
  QD_HIP(hipMalloc((void**)&s->red, doubles * sizeof(double)));
  s->red_cap = doubles;
  return QD_OK;
}

int launch_probabilities(const qd_state* s, double* out_dev) {
  const uint64_t D = uint64_t(s->reg.D);
  constexpr uint64_t kChunk = uint64_t(1) << 30;   // amplitudes per launch (one per thread)
  for (uint64_t o = 0; o < D; o += kChunk) {
    const uint64_t n = std::min(kChunk, D - o);
    const dim3 grid(unsigned((n + 255) / 256));
    if (s->prec == QD_C128)
      hipLaunchKernelGGL((k_probabilities<double>), grid, dim3(256), 0, s->stream, (const double*)s->data + 2 * o,
                         out_dev + o, n);
    else
      hipLaunchKernelGGL((k_probabilities<float>), grid, dim3(256), 0, s->stream, (const float*)s->data + 2 * o,
                         out_dev + o, n);
    QD_HIP(hipGetLastError());
  }
  return QD_OK;
}

int reduce_norm2(const qd_state* cs, double* out) {
  qd_state* s = const_cast<qd_state*>(cs);
  const uint64_t D = uint64_t(s->reg.D);
  const unsigned g = red_grid(D);
  int rc = ensure_red(s, g + 8);
  if (rc) return rc;
  if (s->prec == QD_C128)
    hipLaunchKernelGGL((k_norm_partial<double>), dim3(g), dim3(kRedBlock), 0, s->stream, (const double*)s->data, D, s->red);
  else
    hipLaunchKernelGGL((k_norm_partial<float>), dim3(g), dim3(kRedBlock), 0, s->stream, (const float*)s->data, D, s->red);
  hipLaunchKernelGGL((k_finish<1>), dim3(1), dim3(kRedBlock), 0, s->stream, s->red, g, 1, s->red + g);
  QD_HIP(hipGetLastError());
  QD_HIP(hipMemcpyAsync(out, s->red + g, sizeof(double), hipMemcpyDeviceToHost, s->stream));
  QD_HIP(hipStreamSynchronize(s->stream));
  return QD_OK;
}

int reduce_probabilities_norm2(const qd_state* cs, double* out_dev, double* norm2) {
  qd_state* s = const_cast<qd_state*>(cs);
  const uint64_t D = uint64_t(s->reg.D);
  const unsigned g = red_grid(D);
  int rc = ensure_red(s, g + 8);
  if (rc) return rc;
  if (s->prec == QD_C128)
    hipLaunchKernelGGL((k_probabilities_norm<double>), dim3(g), dim3(kRedBlock), 0, s->stream, (const double*)s->data,
                       out_dev, D, s->red);
  else
    hipLaunchKernelGGL((k_probabilities_norm<float>), dim3(g), dim3(kRedBlock), 0, s->stream, (const float*)s->data,
                       out_dev, D, s->red);
  hipLaunchKernelGGL((k_finish<1>), dim3(1), dim3(kRedBlock), 0, s->stream, s->red, g, 1, s->red + g);
  QD_HIP(hipGetLastError());
  QD_HIP(hipMemcpyAsync(norm2, s->red + g, sizeof(double), hipMemcpyDeviceToHost, s->stream));
  QD_HIP(hipStreamSynchronize(s->stream));
  return QD_OK;
}

// ------------------------------------------------------------------------------------------ state-wide
// elementwise passes: one amplitude (or 16-byte unit) per thread with streaming access, the
// fastest form measured on gfx950 (ahead of grid-stride loops); launches of at most 2^30 items

constexpr uint64_t kElemChunk = uint64_t(1) << 30;

template <typename R>
__global__ __launch_bounds__(256) void k_scale(R* psi_raw, uint64_t n, double f) {
  using C = typename CxR<R>::T;
  C* psi = reinterpret_cast<C*>(psi_raw);
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    C a = ld_stream(psi + i);
    a.x = R(double(a.x) * f);
    a.y = R(double(a.y) * f);
    st_stream(psi + i, a);
  }
}

int scale_state(qd_state* s, double f) {
  const uint64_t D = uint64_t(s->reg.D);
  for (uint64_t o = 0; o < D; o += kElemChunk) {
    const uint64_t n = std::min(kElemChunk, D - o);
    const dim3 grid(unsigned((n + 255) / 256));
    if (s->prec == QD_C128)
      hipLaunchKernelGGL((k_scale<double>), grid, dim3(256), 0, s->stream, (double*)s->data + 2 * o, n, f);
    else
      hipLaunchKernelGGL((k_scale<float>), grid, dim3(256), 0, s->stream, (float*)s->data + 2 * o, n, f);
    QD_HIP(hipGetLastError());
  }
  QD_HIP(hipStreamSynchronize(s->stream));
  return QD_OK;
}

// Scaling by 1/sqrt(||psi||^2) with the squared norm read from device memory (FP64), so the whole
// normalisation stays on the stream: a norm of zero or not finite leaves the state unchanged.
template <typename R>
__global__ __launch_bounds__(256) void k_scale_by_norm(R* psi_raw, uint64_t n, const double* norm2) {
  using C = typename CxR<R>::T;
  C* psi = reinterpret_cast<C*>(psi_raw);
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const double n2 = *norm2;
  if (i < n && n2 > 0.0 && isfinite(n2)) {
    const double f = 1.0 / sqrt(n2);
    C a = ld_stream(psi + i);
    a.x = R(double(a.x) * f);
    a.y = R(double(a.y) * f);
    st_stream(psi + i, a);
  }
}

int normalize_on_device(qd_state* s) {
  const uint64_t D = uint64_t(s->reg.D);
  const unsigned g = red_grid(D);
  int rc = ensure_red(s, g + 8);
  if (rc) return rc;
  if (s->prec == QD_C128)
    hipLaunchKernelGGL((k_norm_partial<double>), dim3(g), dim3(kRedBlock), 0, s->stream, (const double*)s->data, D, s->red);
  else
    hipLaunchKernelGGL((k_norm_partial<float>), dim3(g), dim3(kRedBlock), 0, s->stream, (const float*)s->data, D, s->red);
  hipLaunchKernelGGL((k_finish<1>), dim3(1), dim3(kRedBlock), 0, s->stream, s->red, g, 1, s->red + g);
  QD_HIP(hipGetLastError());
  for (uint64_t o = 0; o < D; o += kElemChunk) {
    const uint64_t n = std::min(kElemChunk, D - o);
    const dim3 grid(unsigned((n + 255) / 256));
    if (s->prec == QD_C128)
      hipLaunchKernelGGL((k_scale_by_norm<double>), grid, dim3(256), 0, s->stream, (double*)s->data + 2 * o, n,
                         (const double*)(s->red + g));
    else
      hipLaunchKernelGGL((k_scale_by_norm<float>), grid, dim3(256), 0, s->stream, (float*)s->data + 2 * o, n,
                         (const double*)(s->red + g));
    QD_HIP(hipGetLastError());
  }
  return QD_OK;
}

// |idx> : amplitude 1 at idx, 0 elsewhere (offset o of the launch's first amplitude)
template <typename R>
__global__ __launch_bounds__(256) void k_fill_basis(R* psi_raw, uint64_t n, uint64_t o, uint64_t idx) {
  using C = typename CxR<R>::T;
  C* psi = reinterpret_cast<C*>(psi_raw);
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    C v;
    v.x = (o + i == idx) ? R(1) : R(0);
    v.y = R(0);
    st_stream(psi + i, v);
  }
}

int launch_fill_basis(qd_state* s, int64_t index) {
  const uint64_t D = uint64_t(s->reg.D);
  for (uint64_t o = 0; o < D; o += kElemChunk) {
    const uint64_t n = std::min(kElemChunk, D - o);
    const dim3 grid(unsigned((n + 255) / 256));
    if (s->prec == QD_C128)
      hipLaunchKernelGGL((k_fill_basis<double>), grid, dim3(256), 0, s->stream, reinterpret_cast<double*>(s->data) + 2 * o,
                         n, o, uint64_t(index));
    else
      hipLaunchKernelGGL((k_fill_basis<float>), grid, dim3(256), 0, s->stream, reinterpret_cast<float*>(s->data) + 2 * o,
                         n, o, uint64_t(index));
    QD_HIP(hipGetLastError());
  }
  return QD_OK;
}

// HBM copy ceiling: one streaming 16-byte load and store per thread (the fastest copy form
// measured on gfx950, ahead of grid-stride loops and of several accesses per thread)
__global__ __launch_bounds__(256) void k_stream_copy(uint4* __restrict__ dst, const uint4* __restrict__ src, uint64_t n16) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n16) st_stream(dst + i, ld_stream(src + i));
}

int launch_stream_copy(void* dst, const void* src, int64_t bytes, hipStream_t st) {
  const uint64_t n16 = uint64_t(bytes) / 16;
  for (uint64_t o = 0; o < n16; o += kElemChunk) {
    const uint64_t n = std::min(kElemChunk, n16 - o);
    hipLaunchKernelGGL(k_stream_copy, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<uint4*>(dst) + o, reinterpret_cast<const uint4*>(src) + o, n);
    QD_HIP(hipGetLastError());
  }
  return QD_OK;
}

// ------------------------------------------------------------------------------------------ no-allocation norm
// The partials of the squared-norm reduction of a caller that cannot allocate live in one
// file-scope device array per GPU, sized for the largest reduction grid. Its device address is
// looked up once per device (with that device current) and used for every launch; the host-side
// name of the array is never passed to a kernel.
constexpr int kStaticRedDoubles = kRedMaxGrid;   // 16 KiB per GPU
constexpr int kStaticMaxDevices = 64;
static __device__ __align__(256) double scratch[kStaticRedDoubles];

static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kStaticMaxDevices] = {};

static int static_scratch(int device, double** out) {
  if (device < 0 || device >= kStaticMaxDevices) return fail(QD_EDEVICE, "device id beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    QD_HIP(hipGetDevice(&cur));
    if (cur != device) QD_HIP(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) QD_HIP(hipSetDevice(cur));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(QD_EDEVICE, "no device address for the static scratch array");
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[device];
  return QD_OK;
}

int reduce_norm2_noalloc(const qd_state* s, double* out_dev) {
  const uint64_t D = uint64_t(s->reg.D);
  const unsigned g = red_grid(D);
  if (g > unsigned(kStaticRedDoubles))
    return fail(QD_EINVAL, "reduction grid exceeds the static scratch array (2048 partials)");
  double* part = nullptr;
  int rc = static_scratch(s->device, &part);
  if (rc) return rc;
  // every workgroup writes its own partial, so nothing needs clearing between calls
  if (s->prec == QD_C128)
    hipLaunchKernelGGL((k_norm_partial<double>), dim3(g), dim3(kRedBlock), 0, s->stream, (const double*)s->data, D, part);
  else
    hipLaunchKernelGGL((k_norm_partial<float>), dim3(g), dim3(kRedBlock), 0, s->stream, (const float*)s->data, D, part);
  hipLaunchKernelGGL((k_finish<1>), dim3(1), dim3(kRedBlock), 0, s->stream, part, g, 1, out_dev);
  QD_HIP(hipGetLastError());
  return QD_OK;
}

int reduce_compare(const qd_state* ref, const qd_state* cs, double* max_abs, double* fid, double* drift,
                   double* norm2, double* fid_norm) {
  qd_state* s = const_cast<qd_state*>(cs);
  // the reference must be complete before s's stream reads it
  if (ref->stream != s->stream) QD_HIP(hipStreamSynchronize(ref->stream));
  const uint64_t D = uint64_t(s->reg.D);
  const unsigned g = red_grid(D);
  int rc = ensure_red(s, 4 * size_t(g) + 8);
  if (rc) return rc;
  if (s->prec == QD_C128)
    hipLaunchKernelGGL((k_compare_partial<double>), dim3(g), dim3(kRedBlock), 0, s->stream, (const double*)ref->data,
                       (const double*)s->data, D, s->red);
  else
    hipLaunchKernelGGL((k_compare_partial<float>), dim3(g), dim3(kRedBlock), 0, s->stream, (const double*)ref->data,
                       (const float*)s->data, D, s->red);
  hipLaunchKernelGGL((k_finish<4>), dim3(1), dim3(kRedBlock), 0, s->stream, s->red, g, 3, s->red + 4 * size_t(g));
  QD_HIP(hipGetLastError());
  double h[4];
  QD_HIP(hipMemcpyAsync(h, s->red + 4 * size_t(g), 4 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  QD_HIP(hipStreamSynchronize(s->stream));
  const double ov = h[0] * h[0] + h[1] * h[1];
  if (max_abs) *max_abs = h[3];
  if (fid) *fid = 1.0 - ov;
  if (drift) *drift = std::fabs(h[2] - 1.0);
  if (norm2) *norm2 = h[2];
  if (fid_norm) *fid_norm = h[2] > 0.0 ? 1.0 - ov / h[2] : 1.0;
  return QD_OK;
}

}  // namespace qd
