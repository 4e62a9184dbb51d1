// Density matrices and noise channels. The paper keeps states as vectors and names density
// matrices (Sec. 3.3) and noise models (Sec. 7) as the next representations; a channel on qudits
// of dimensions (d_1..d_k) has Kraus matrices of the size a gate on them has (Sec. 3.1).
//
// A density matrix rho over a register of n qudits (D = prod d_i) is stored as a state over the
// doubled register dims ++ dims: row qudits 0..n-1, column qudits n..2n-1, so element (x, y) sits
// at flat index x * D + y (row-major). With this layout
//   * a gate G maps rho -> G rho G^dagger, i.e. G on the row qudits and conj(G) on the column
//     qudits. With G embedded on its targets and controls (dimension d_G = d_T x d_C), a diagonal
//     gate with d_G <= kOnePass and an uncontrolled gate with d_T <= kOnePass are one pass of
//     G (x) conj(G) over (T, C, T + n, C + n); every other gate (in particular every controlled gate
//     that is not diagonal) takes two passes: U on T with its controls, conj(U) on T + n with the
//     shifted controls, each over the elements whose control digits match;
//   * a channel with Kraus operators K_1..K_r maps rho -> sum_k K_k rho K_k^dagger, one pass of the
//     superoperator S = sum_k K_k (x) conj(K_k) over (T, T + n);
//   * consecutive operations whose targets and controls together span qudits Sq of dimension
//     <= kFuseGroup are composed on the host into one superoperator on (Sq, Sq + n), each embedded
//     on Sq, and applied in one pass.
// Both run through the library's gate kernels (HBM-bound passes over the D^2 elements). The
// readouts here (outer product, diagonal, trace, <psi|rho|psi>) are HBM-bound kernels of their own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "qd_internal.h"
#include "qd_stream.h"

namespace qd {
namespace dm {

constexpr int kBlock = 256;
// d_G (targets x controls) up to which a gate is one pass of G (x) conj(G). An uncontrolled gate on
// d_T <= 4 gives a superoperator of at most 16 x 16, one pass that beats two full ones. A controlled
// gate (d_G >= 4) that is not diagonal stays at two passes: each touches only the elements whose
// control digits match (2 x 0.36 ms with a qubit control on 1.07e8 elements), while its 16 x 16
// superoperator needs a full pass of more work per element (0.66-0.71 ms measured for the dense and
// the permutation cases). Diagonal superoperators cost one elementwise pass, so a diagonal gate is
// one pass whenever d_G <= 4.
constexpr int kOnePass = 4;
constexpr int kMaxChannelDim = 32;    // d_T of a channel (its superoperator is d_T^2 x d_T^2 <= 1024)
constexpr int kFuseGroup = 4;         // dimension of the qudits a run of operations touches, up to which it is one pass
constexpr int kRedGrid = 1024;

template <typename R> struct Cx;
template <> struct Cx<double> { using T = double2; };
template <> struct Cx<float> { using T = float2; };

// rho[x, y] = psi[x] conj(psi[y]); one column index y per thread, rows x strided over grid.y
template <typename R>
__global__ __launch_bounds__(kBlock) void k_outer(const R* __restrict__ psi_raw, R* __restrict__ rho_raw, uint64_t D) {
  using C = typename Cx<R>::T;
  const C* psi = reinterpret_cast<const C*>(psi_raw);
  C* rho = reinterpret_cast<C*>(rho_raw);
  const uint64_t y = uint64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (y >= D) return;
  const C b = psi[y];
  const double br = double(b.x), bi = -double(b.y);
  for (uint64_t x = blockIdx.y; x < D; x += gridDim.y) {
    const C a = psi[x];
    const double ar = double(a.x), ai = double(a.y);
    C v;
    v.x = R(ar * br - ai * bi);
    v.y = R(ar * bi + ai * br);
    st_stream(rho + x * D + y, v);
  }
}

// out[x] = Re rho[x, x]
template <typename R>
__global__ __launch_bounds__(kBlock) void k_diag(const R* __restrict__ rho_raw, uint64_t D, double* __restrict__ out) {
  using C = typename Cx<R>::T;
  const C* rho = reinterpret_cast<const C*>(rho_raw);
  const uint64_t x = uint64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (x < D) out[x] = double(rho[x * (D + 1)].x);
}

// fixed-order block sum of NV values per thread into part[blockIdx.x * NV + q]
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* part) {
  __shared__ double sh[NV][kBlock];
#pragma unroll
  for (int q = 0; q < NV; ++q) sh[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w)
#pragma unroll
      for (int q = 0; q < NV; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) part[blockIdx.x * NV + q] = sh[q][0];
}

// trace: partial sums of the diagonal (re, im) over a fixed grid
template <typename R>
__global__ __launch_bounds__(kBlock) void k_trace_part(const R* __restrict__ rho_raw, uint64_t D, double* __restrict__ part) {
  using C = typename Cx<R>::T;
  const C* rho = reinterpret_cast<const C*>(rho_raw);
  double v[2] = {0.0, 0.0};
  for (uint64_t x = uint64_t(blockIdx.x) * kBlock + threadIdx.x; x < D; x += uint64_t(gridDim.x) * kBlock) {
    const C a = rho[x * (D + 1)];
    v[0] += double(a.x);
    v[1] += double(a.y);
  }
  block_sum<2>(v, part);
}

// <psi|rho|psi> = sum_x conj(psi_x) sum_y rho_xy psi_y: each workgroup takes whole rows (row x of
// workgroup b: x = b, b + grid, ...), its threads stride over y with coalesced streaming reads
template <typename R>
__global__ __launch_bounds__(kBlock) void k_fidelity_part(const R* __restrict__ rho_raw, const R* __restrict__ psi_raw,
                                                          uint64_t D, double* __restrict__ part) {
  using C = typename Cx<R>::T;
  const C* rho = reinterpret_cast<const C*>(rho_raw);
  const C* psi = reinterpret_cast<const C*>(psi_raw);
  double v[2] = {0.0, 0.0};
  for (uint64_t x = blockIdx.x; x < D; x += gridDim.x) {
    double rr = 0.0, ri = 0.0;
    const C* row = rho + x * D;
    for (uint64_t y = threadIdx.x; y < D; y += kBlock) {
      const C a = ld_stream(row + y);
      const C b = psi[y];
      rr += double(a.x) * double(b.x) - double(a.y) * double(b.y);
      ri += double(a.x) * double(b.y) + double(a.y) * double(b.x);
    }
    const C p = psi[x];
    // conj(psi_x) * (rr + i ri)
    v[0] += double(p.x) * rr + double(p.y) * ri;
    v[1] += double(p.x) * ri - double(p.y) * rr;
  }
  block_sum<2>(v, part);
}

static unsigned red_grid(uint64_t D) {
  return unsigned(std::max<uint64_t>(1, std::min<uint64_t>(kRedGrid, (D + kBlock - 1) / kBlock)));
}

// sum the NV partials of g workgroups on the host in a fixed order
static int finish(qd_state* s, double* part, unsigned g, int nv, double* out) {
  std::vector<double> h(size_t(g) * nv);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  (void)hipFree(part);
  if (e != hipSuccess) return hip_fail(e, "density reduction");
  for (int q = 0; q < nv; ++q) {
    double acc = 0.0;
    for (unsigned b = 0; b < g; ++b) acc += h[size_t(b) * nv + q];
    out[q] = acc;
  }
  return QD_OK;
}

static bool same_register(const qd_state* rho, const qd_state* psi) {
  const int n = rho->dens_n;
  if (psi->dens_n || psi->reg.n != n) return false;
  for (int i = 0; i < n; ++i)
    if (psi->reg.dims[i] != rho->reg.dims[i]) return false;
  return true;
}

// validated channel: the superoperator S = sum_k K_k (x) conj(K_k), (d_T^2 x d_T^2, interleaved)
static std::vector<double> superoperator(const double* kraus, int32_t nk, int dT) {
  const int N = dT * dT;
  std::vector<double> S(2 * size_t(N) * N, 0.0);
  for (int k = 0; k < nk; ++k) {
    const double* K = kraus + 2 * size_t(k) * dT * dT;
    for (int a = 0; a < dT; ++a)
      for (int b = 0; b < dT; ++b)
        for (int c = 0; c < dT; ++c)
          for (int d = 0; d < dT; ++d) {
            // row (a, b), column (c, d): K[a][c] * conj(K[b][d])
            const double xr = K[2 * (a * dT + c)], xi = K[2 * (a * dT + c) + 1];
            const double yr = K[2 * (b * dT + d)], yi = -K[2 * (b * dT + d) + 1];
            const size_t o = 2 * (size_t(a * dT + b) * N + size_t(c * dT + d));
            S[o] += xr * yr - xi * yi;
            S[o + 1] += xr * yi + xi * yr;
          }
  }
  return S;
}

// The matrices of an operation on the qudit list Sq (first most significant): a gate's controlled
// unitary (U on its targets where its controls hold their values, the identity elsewhere) or each
// Kraus matrix of a channel, times the identity on the other qudits of Sq.
static std::vector<double> embed_on(const Register& phys, const qd_density_op& o, const std::vector<int>& Sq) {
  const int ns = int(Sq.size());
  int dS = 1, dT = 1;
  for (int q : Sq) dS *= phys.dims[q];
  for (int j = 0; j < o.k; ++j) dT *= phys.dims[o.targets[j]];
  const int nk = o.kind == QD_OP_GATE ? 1 : o.nk;
  const int m = o.kind == QD_OP_GATE ? o.m : 0;
  std::vector<int> tpos(o.k), tmul(o.k), cpos(m);
  auto pos_of = [&](int q) { return int(std::find(Sq.begin(), Sq.end(), q) - Sq.begin()); };
  for (int j = o.k - 1, mul = 1; j >= 0; --j) {
    tpos[j] = pos_of(o.targets[j]);
    tmul[j] = mul;
    mul *= phys.dims[o.targets[j]];
  }
  for (int j = 0; j < m; ++j) cpos[j] = pos_of(o.controls[j]);
  std::vector<char> is_t(ns, 0);
  for (int j = 0; j < o.k; ++j) is_t[tpos[j]] = 1;
  std::vector<double> W(2 * size_t(nk) * dS * dS, 0.0);
  std::vector<int> dx(ns), dy(ns);
  for (int x = 0; x < dS; ++x)
    for (int y = 0; y < dS; ++y) {
      for (int s = ns - 1, rx = x, ry = y; s >= 0; --s) {
        dx[s] = rx % phys.dims[Sq[s]];
        dy[s] = ry % phys.dims[Sq[s]];
        rx /= phys.dims[Sq[s]];
        ry /= phys.dims[Sq[s]];
      }
      bool same = true;                   // every digit the operation does not act on is kept
      for (int s = 0; s < ns; ++s) same = same && (is_t[s] || dx[s] == dy[s]);
      if (!same) continue;
      bool on = true;
      for (int j = 0; j < m; ++j) on = on && dy[cpos[j]] == o.control_values[j];
      int tx = 0, ty = 0;
      for (int j = 0; j < o.k; ++j) {
        tx += dx[tpos[j]] * tmul[j];
        ty += dy[tpos[j]] * tmul[j];
      }
      for (int kk = 0; kk < nk; ++kk) {
        const size_t w = 2 * (size_t(kk) * dS * dS + size_t(x) * dS + y);
        if (on) {
          const double* K = o.mats + 2 * size_t(kk) * dT * dT;
          W[w] = K[2 * (tx * dT + ty)];
          W[w + 1] = K[2 * (tx * dT + ty) + 1];
        } else if (tx == ty) {
          W[w] = 1.0;
        }
      }
    }
  return W;
}

}  // namespace dm
}  // namespace qd

using namespace qd;
using namespace qd::dm;

extern "C" {

int qd_density_init(const int32_t* dims, int32_t n, int32_t prec, void* hip_stream, qd_state** out) {
  if (!dims || !out) return fail(QD_EINVAL, "null argument");
  if (n < 1 || 2 * n > QD_MAX_QUDITS) return fail(QD_EINVAL, "a density matrix holds 1..32 qudits");
  std::vector<int32_t> d2(dims, dims + n);
  d2.insert(d2.end(), dims, dims + n);
  int rc = qd_state_init(d2.data(), 2 * n, prec, hip_stream, out);   // |0..0><0..0|: element 0 is 1
  if (rc) return rc;
  (*out)->dens_n = n;
  return QD_OK;
}

int qd_density_from_state(qd_state* rho, const qd_state* psi) {
  if (!rho || !psi) return fail(QD_EINVAL, "null argument");
  if (!rho->dens_n) return fail(QD_EINVAL, "not a density matrix");
  if (!same_register(rho, psi)) return fail(QD_EDIM, "the state's register differs from the density matrix's");
  if (psi->prec != rho->prec) return fail(QD_EINVAL, "the state and the density matrix differ in precision");
  const uint64_t D = uint64_t(psi->reg.D);
  // psi may be written on its own stream: finish it before this stream reads it
  QD_HIP(hipStreamSynchronize(psi->stream));
  const dim3 grid(unsigned((D + kBlock - 1) / kBlock), unsigned(std::min<uint64_t>(D, 65535)));
  if (rho->prec == QD_C128)
    hipLaunchKernelGGL(k_outer<double>, grid, dim3(kBlock), 0, rho->stream, (const double*)psi->data, (double*)rho->data, D);
  else
    hipLaunchKernelGGL(k_outer<float>, grid, dim3(kBlock), 0, rho->stream, (const float*)psi->data, (float*)rho->data, D);
  QD_HIP(hipGetLastError());
  return QD_OK;
}

int qd_density_apply_gate(qd_state* rho, const int32_t* targets, int32_t k, const int32_t* controls,
                          const int32_t* control_values, int32_t m, const double* U, uint32_t flags) {
  if (!rho) return fail(QD_EINVAL, "null state");
  if (!rho->dens_n) return fail(QD_EINVAL, "not a density matrix");
  const int n = rho->dens_n;
  // validate against the physical register (targets and controls must be row qudits)
  Register phys{};
  int rc = make_register(rho->reg.dims, n, &phys);
  if (rc) return rc;
  rc = validate_gate(phys, targets, k, controls, control_values, m, U, flags);
  if (rc) return rc;
  int dT = 1;
  for (int j = 0; j < k; ++j) dT *= phys.dims[targets[j]];
  int dC = 1;
  for (int j = 0; j < m; ++j) dC *= phys.dims[controls[j]];
  const int dG = dT * dC;                 // the gate embedded on (targets, controls)
  const uint32_t skip = flags | QD_FLAG_SKIP_UNITARY_CHECK;
  const int cls = classify(U, dT);
  const bool one_pass = cls == QD_CLASS_DIAGONAL ? dG <= kOnePass : (m == 0 && dT <= kOnePass);
  if (one_pass) {
    // one pass of G (x) conj(G) over (T, C, T + n, C + n), G[(t, c), (t', c')] = delta(c, c') times
    // U[t][t'] when the control digits c hold the control values, else delta(t, t')
    std::vector<double> G(2 * size_t(dG) * dG, 0.0);
    int vidx = 0;                          // local index of the control values (first control most significant)
    for (int j = 0; j < m; ++j) vidx = vidx * phys.dims[controls[j]] + control_values[j];
    for (int c = 0; c < dC; ++c)
      for (int t = 0; t < dT; ++t)
        for (int t1 = 0; t1 < dT; ++t1) {
          const size_t o = 2 * (size_t(t * dC + c) * dG + size_t(t1 * dC + c));
          if (c == vidx) {
            G[o] = U[2 * (t * dT + t1)];
            G[o + 1] = U[2 * (t * dT + t1) + 1];
          } else if (t == t1) {
            G[o] = 1.0;
          }
        }
    const int N = dG * dG;
    std::vector<double> M(2 * size_t(N) * N);
    for (int a = 0; a < dG; ++a)
      for (int b = 0; b < dG; ++b)
        for (int c = 0; c < dG; ++c)
          for (int d = 0; d < dG; ++d) {
            // element ((a, b), (c, d)) = G[a][c] conj(G[b][d])
            const double xr = G[2 * (a * dG + c)], xi = G[2 * (a * dG + c) + 1];
            const double yr = G[2 * (b * dG + d)], yi = -G[2 * (b * dG + d) + 1];
            const size_t o = 2 * (size_t(a * dG + b) * N + size_t(c * dG + d));
            M[o] = xr * yr - xi * yi;
            M[o + 1] = xr * yi + xi * yr;
          }
    std::vector<int32_t> q(targets, targets + k);
    q.insert(q.end(), controls, controls + m);
    for (int j = 0; j < k + m; ++j) q.push_back(q[size_t(j)] + n);
    return qd_apply_gate_ex(rho, q.data(), 2 * (k + m), nullptr, nullptr, 0, M.data(), skip);
  }
  std::vector<int32_t> t2(targets, targets + k), c2;
  for (int j = 0; j < k; ++j) t2.push_back(targets[j] + n);
  rc = qd_apply_gate_ex(rho, targets, k, controls, control_values, m, U, skip);
  if (rc) return rc;
  std::vector<double> Uc(U, U + 2 * size_t(dT) * dT);
  for (size_t i = 1; i < Uc.size(); i += 2) Uc[i] = -Uc[i];
  for (int j = 0; j < m; ++j) c2.push_back(controls[j] + n);
  return qd_apply_gate_ex(rho, t2.data() + k, k, m ? c2.data() : nullptr, control_values, m, Uc.data(), skip);
}

int qd_density_apply_channel(qd_state* rho, const int32_t* targets, int32_t k, const double* kraus, int32_t nk,
                             uint32_t flags) {
  if (!rho) return fail(QD_EINVAL, "null state");
  if (!rho->dens_n) return fail(QD_EINVAL, "not a density matrix");
  if (!kraus || nk < 1) return fail(QD_EINVAL, "a channel needs at least one Kraus operator");
  const int n = rho->dens_n;
  Register phys{};
  int rc = make_register(rho->reg.dims, n, &phys);
  if (rc) return rc;
  if (!targets || k < 1 || k > n) return fail(QD_EINVAL, "bad target list");
  bool used[QD_MAX_QUDITS] = {};
  int dT = 1;
  for (int j = 0; j < k; ++j) {
    if (targets[j] < 0 || targets[j] >= n) return fail(QD_EINVAL, "target out of range");
    if (used[targets[j]]) return fail(QD_EINVAL, "duplicate target");
    used[targets[j]] = true;
    dT *= phys.dims[targets[j]];
    if (dT > kMaxChannelDim) return fail(QD_EDIM, "channel dimension d_T exceeds 32");
  }
  const size_t kk = size_t(dT) * dT;
  for (size_t i = 0; i < 2 * kk * size_t(nk); ++i)
    if (!std::isfinite(kraus[i])) return fail(QD_ENOTUNITARY, "a Kraus operator has a NaN or Inf entry");
  if (!(flags & QD_FLAG_SKIP_UNITARY_CHECK)) {
    // trace preservation: max |sum_k K_k^dagger K_k - I| <= 1e-10
    for (int i = 0; i < dT; ++i)
      for (int j = 0; j < dT; ++j) {
        double re = 0.0, im = 0.0;
        for (int q = 0; q < nk; ++q) {
          const double* K = kraus + 2 * kk * size_t(q);
          for (int l = 0; l < dT; ++l) {
            const double ar = K[2 * (l * dT + i)], ai = -K[2 * (l * dT + i) + 1];
            const double br = K[2 * (l * dT + j)], bi = K[2 * (l * dT + j) + 1];
            re += ar * br - ai * bi;
            im += ar * bi + ai * br;
          }
        }
        if (i == j) re -= 1.0;
        if (std::sqrt(re * re + im * im) > 1e-10) return fail(QD_ENOTUNITARY, "Kraus operators do not sum to the identity");
      }
  }
  std::vector<int32_t> t2(targets, targets + k);
  for (int j = 0; j < k; ++j) t2.push_back(targets[j] + n);
  const std::vector<double> S = superoperator(kraus, nk, dT);
  return qd_apply_gate_ex(rho, t2.data(), 2 * k, nullptr, nullptr, 0, S.data(), QD_FLAG_SKIP_UNITARY_CHECK);
}

int qd_channel_kraus(int32_t kind, int32_t d, double p, double* out, int32_t cap, int32_t* nk) {
  if (!nk) return fail(QD_EINVAL, "null count");
  if (d < 2 || d > QD_MAX_RADIX) return fail(QD_EDIM, "dimension must be 2..256");
  if (!(p >= 0.0 && p <= 1.0)) return fail(QD_EINVAL, "probability must be in [0, 1]");
  const int count = kind == QD_CHANNEL_DEPOLARIZING ? d * d : kind == QD_CHANNEL_DEPHASING || kind == QD_CHANNEL_AMPLITUDE_DAMPING ? d : -1;
  if (count < 0) return fail(QD_EINVAL, "unknown channel kind");
  *nk = count;
  if (!out) return QD_OK;
  if (cap < count) return fail(QD_EINVAL, "output holds fewer Kraus operators than the channel has");
  const size_t dd = size_t(d) * d;
  std::fill(out, out + 2 * dd * size_t(count), 0.0);
  auto at = [&](int q, int r, int c) { return out + 2 * (dd * size_t(q) + size_t(r) * d + c); };
  std::vector<double> Z(2 * dd), X(2 * dd);
  if (kind == QD_CHANNEL_AMPLITUDE_DAMPING) {
    at(0, 0, 0)[0] = 1.0;
    for (int j = 1; j < d; ++j) {
      at(0, j, j)[0] = std::sqrt(1.0 - p);
      at(j, j - 1, j)[0] = std::sqrt(p);
    }
    return QD_OK;
  }
  // Z^b: diag omega^{b j}, X^a: |j> -> |j + a mod d>, built from the library's named gates
  int rc = qd_gate_matrix(QD_GATE_Z, d, 0, Z.data());
  if (rc) return rc;
  if (kind == QD_CHANNEL_DEPHASING) {
    for (int b = 0; b < d; ++b) {
      const double w = b == 0 ? std::sqrt(1.0 - p) : std::sqrt(p / (d - 1));
      for (int j = 0; j < d; ++j) {
        // omega^{b j} = (Z[j][j])^b, taken from the reduced exponent b j mod d
        const int e = (b * j) % d;
        // Z[e][e] holds omega^e
        at(b, j, j)[0] = w * Z[2 * (size_t(e) * d + e)];
        at(b, j, j)[1] = w * Z[2 * (size_t(e) * d + e) + 1];
      }
    }
    return QD_OK;
  }
  // depolarizing: K_ab = w_ab X^a Z^b, (X^a Z^b)[r][c] = omega^{b c} when r = c + a mod d
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      const double w = (a == 0 && b == 0) ? std::sqrt(1.0 - p + p / (double(d) * d)) : std::sqrt(p / (double(d) * d));
      const int q = a * d + b;
      for (int c = 0; c < d; ++c) {
        const int r = (c + a) % d, e = (b * c) % d;
        at(q, r, c)[0] = w * Z[2 * (size_t(e) * d + e)];
        at(q, r, c)[1] = w * Z[2 * (size_t(e) * d + e) + 1];
      }
    }
  return QD_OK;
}

int qd_density_apply_ops(qd_state* rho, const qd_density_op* ops, int32_t count, uint32_t flags) {
  if (!rho) return fail(QD_EINVAL, "null state");
  if (!rho->dens_n) return fail(QD_EINVAL, "not a density matrix");
  if (count < 0 || (count > 0 && !ops)) return fail(QD_EINVAL, "null operations or negative count");
  const int n = rho->dens_n;
  Register phys{};
  int rc = make_register(rho->reg.dims, n, &phys);
  if (rc) return rc;
  // validate everything before any device work
  for (int32_t i = 0; i < count; ++i) {
    const qd_density_op& o = ops[i];
    if (o.kind == QD_OP_GATE) {
      if (o.nk != 1 || !o.mats) return fail(QD_EINVAL, "a gate operation carries one matrix");
      rc = validate_gate(phys, o.targets, o.k, o.controls, o.control_values, o.m, o.mats, flags);
    } else if (o.kind == QD_OP_CHANNEL) {
      if (o.m != 0) return fail(QD_EINVAL, "a channel operation has no controls");
      if (!o.mats || o.nk < 1) return fail(QD_EINVAL, "a channel needs at least one Kraus operator");
      // reuse the channel's own checks on a scratch-free path: targets, d_T and completeness
      if (!o.targets || o.k < 1 || o.k > n) return fail(QD_EINVAL, "bad target list");
      bool used[QD_MAX_QUDITS] = {};
      int dT = 1;
      for (int j = 0; j < o.k; ++j) {
        if (o.targets[j] < 0 || o.targets[j] >= n || used[o.targets[j]]) return fail(QD_EINVAL, "bad target list");
        used[o.targets[j]] = true;
        dT *= phys.dims[o.targets[j]];
        if (dT > kMaxChannelDim) return fail(QD_EDIM, "channel dimension d_T exceeds 32");
      }
      const size_t kk = size_t(dT) * dT;
      for (size_t q = 0; q < 2 * kk * size_t(o.nk); ++q)
        if (!std::isfinite(o.mats[q])) return fail(QD_ENOTUNITARY, "a Kraus operator has a NaN or Inf entry");
      if (!(flags & QD_FLAG_SKIP_UNITARY_CHECK)) {
        for (int a = 0; a < dT; ++a)
          for (int b = 0; b < dT; ++b) {
            double re = 0.0, im = 0.0;
            for (int q = 0; q < o.nk; ++q) {
              const double* K = o.mats + 2 * kk * size_t(q);
              for (int l = 0; l < dT; ++l) {
                const double ar = K[2 * (l * dT + a)], ai = -K[2 * (l * dT + a) + 1];
                const double br = K[2 * (l * dT + b)], bi = K[2 * (l * dT + b) + 1];
                re += ar * br - ai * bi;
                im += ar * bi + ai * br;
              }
            }
            if (a == b) re -= 1.0;
            if (std::sqrt(re * re + im * im) > 1e-10) return fail(QD_ENOTUNITARY, "Kraus operators do not sum to the identity");
          }
      }
      rc = QD_OK;
    } else {
      return fail(QD_EINVAL, "unknown operation kind");
    }
    if (rc) return rc;
  }
  const uint32_t skip = flags | QD_FLAG_SKIP_UNITARY_CHECK;
  // the sorted union of a list of qudits and an operation's targets and controls
  auto with_support = [&](std::vector<int> sq, const qd_density_op& o) {
    for (int j = 0; j < o.k; ++j) sq.push_back(o.targets[j]);
    if (o.kind == QD_OP_GATE)
      for (int j = 0; j < o.m; ++j) sq.push_back(o.controls[j]);
    std::sort(sq.begin(), sq.end());
    sq.erase(std::unique(sq.begin(), sq.end()), sq.end());
    return sq;
  };
  auto dim_of_set = [&](const std::vector<int>& sq) {
    int d = 1;
    for (int q : sq) d *= phys.dims[q];
    return d;
  };
  int32_t i = 0;
  while (i < count) {
    const qd_density_op& o = ops[i];
    std::vector<int> Sq = with_support({}, o);
    int32_t e = i + 1;
    if (dim_of_set(Sq) <= kFuseGroup)
      while (e < count) {
        std::vector<int> U2 = with_support(Sq, ops[e]);
        if (dim_of_set(U2) > kFuseGroup) break;
        Sq.swap(U2);
        ++e;
      }
    if (e - i == 1) {
      rc = o.kind == QD_OP_GATE
               ? qd_density_apply_gate(rho, o.targets, o.k, o.controls, o.control_values, o.m, o.mats, skip)
               : qd_density_apply_channel(rho, o.targets, o.k, o.mats, o.nk, skip);
      if (rc) return rc;
      i = e;
      continue;
    }
    // compose S = S_{e-1} ... S_i in FP64 on the run's qudits Sq: a gate contributes W (x) conj(W),
    // a channel sum_k W_k (x) conj(W_k), with W its matrices embedded on Sq
    const int dT = dim_of_set(Sq), N = dT * dT;
    std::vector<double> S(2 * size_t(N) * N, 0.0), T, P(2 * size_t(N) * N);
    for (int r = 0; r < N; ++r) S[2 * (size_t(r) * N + r)] = 1.0;
    for (int32_t q = i; q < e; ++q) {
      const qd_density_op& g = ops[q];
      const std::vector<double> W = embed_on(phys, g, Sq);
      T = superoperator(W.data(), g.kind == QD_OP_GATE ? 1 : g.nk, dT);
      // P = T * S
      for (int r = 0; r < N; ++r)
        for (int c = 0; c < N; ++c) {
          double re = 0.0, im = 0.0;
          for (int l = 0; l < N; ++l) {
            const double ar = T[2 * (size_t(r) * N + l)], ai = T[2 * (size_t(r) * N + l) + 1];
            const double br = S[2 * (size_t(l) * N + c)], bi = S[2 * (size_t(l) * N + c) + 1];
            re += ar * br - ai * bi;
            im += ar * bi + ai * br;
          }
          P[2 * (size_t(r) * N + c)] = re;
          P[2 * (size_t(r) * N + c) + 1] = im;
        }
      S.swap(P);
    }
    std::vector<int32_t> t2(Sq.begin(), Sq.end());
    for (int q : Sq) t2.push_back(q + n);
    rc = qd_apply_gate_ex(rho, t2.data(), int32_t(t2.size()), nullptr, nullptr, 0, S.data(), QD_FLAG_SKIP_UNITARY_CHECK);
    if (rc) return rc;
    i = e;
  }
  return QD_OK;
}

int qd_density_trace(qd_state* rho, double* re, double* im) {
  if (!rho || !re || !im) return fail(QD_EINVAL, "null argument");
  if (!rho->dens_n) return fail(QD_EINVAL, "not a density matrix");
  Register phys{};
  int rc = make_register(rho->reg.dims, rho->dens_n, &phys);
  if (rc) return rc;
  const uint64_t Dp = uint64_t(phys.D);
  const unsigned g = red_grid(Dp);
  double* part = nullptr;
  QD_HIP(hipMalloc((void**)&part, size_t(g) * 2 * sizeof(double)));
  if (rho->prec == QD_C128)
    hipLaunchKernelGGL(k_trace_part<double>, dim3(g), dim3(kBlock), 0, rho->stream, (const double*)rho->data, Dp, part);
  else
    hipLaunchKernelGGL(k_trace_part<float>, dim3(g), dim3(kBlock), 0, rho->stream, (const float*)rho->data, Dp, part);
  double o[2];
  rc = finish(rho, part, g, 2, o);
  if (rc) return rc;
  *re = o[0];
  *im = o[1];
  return QD_OK;
}

int qd_density_probabilities(qd_state* rho, double* out, int32_t out_is_device) {
  if (!rho || !out) return fail(QD_EINVAL, "null argument");
  if (!rho->dens_n) return fail(QD_EINVAL, "not a density matrix");
  Register phys{};
  int rc = make_register(rho->reg.dims, rho->dens_n, &phys);
  if (rc) return rc;
  const uint64_t D = uint64_t(phys.D);
  double* dst = out;
  if (!out_is_device) QD_HIP(hipMalloc((void**)&dst, D * sizeof(double)));
  const dim3 grid(unsigned((D + kBlock - 1) / kBlock));
  if (rho->prec == QD_C128)
    hipLaunchKernelGGL(k_diag<double>, grid, dim3(kBlock), 0, rho->stream, (const double*)rho->data, D, dst);
  else
    hipLaunchKernelGGL(k_diag<float>, grid, dim3(kBlock), 0, rho->stream, (const float*)rho->data, D, dst);
  hipError_t e = hipGetLastError();
  if (!out_is_device) {
    if (e == hipSuccess) e = hipMemcpyAsync(out, dst, D * sizeof(double), hipMemcpyDeviceToHost, rho->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(rho->stream);
    (void)hipFree(dst);
  } else if (e == hipSuccess) {
    e = hipStreamSynchronize(rho->stream);
  }
  if (e != hipSuccess) return hip_fail(e, "qd_density_probabilities");
  return QD_OK;
}

int qd_density_purity(qd_state* rho, double* out) {
  if (!rho || !out) return fail(QD_EINVAL, "null argument");
  if (!rho->dens_n) return fail(QD_EINVAL, "not a density matrix");
  return reduce_norm2(rho, out);     // tr(rho^2) = sum |rho_xy|^2 for a Hermitian rho
}

int qd_density_fidelity(qd_state* rho, const qd_state* psi, double* out) {
  if (!rho || !psi || !out) return fail(QD_EINVAL, "null argument");
  if (!rho->dens_n) return fail(QD_EINVAL, "not a density matrix");
  if (!same_register(rho, psi)) return fail(QD_EDIM, "the state's register differs from the density matrix's");
  if (psi->prec != rho->prec) return fail(QD_EINVAL, "the state and the density matrix differ in precision");
  QD_HIP(hipStreamSynchronize(psi->stream));
  const uint64_t D = uint64_t(psi->reg.D);
  const unsigned g = unsigned(std::max<uint64_t>(1, std::min<uint64_t>(kRedGrid, D)));
  double* part = nullptr;
  QD_HIP(hipMalloc((void**)&part, size_t(g) * 2 * sizeof(double)));
  if (rho->prec == QD_C128)
    hipLaunchKernelGGL(k_fidelity_part<double>, dim3(g), dim3(kBlock), 0, rho->stream, (const double*)rho->data,
                       (const double*)psi->data, D, part);
  else
    hipLaunchKernelGGL(k_fidelity_part<float>, dim3(g), dim3(kBlock), 0, rho->stream, (const float*)rho->data,
                       (const float*)psi->data, D, part);
  double o[2];
  int rc = finish(rho, part, g, 2, o);
  if (rc) return rc;
  *out = o[0];
  return QD_OK;
}

int qd_density_size(const qd_state* rho, int32_t* n_qudits) {
  if (!rho || !n_qudits) return fail(QD_EINVAL, "null argument");
  *n_qudits = rho->dens_n;
  return QD_OK;
}

}  // extern "C"
