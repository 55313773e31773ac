// Host side of the DG Maxwell curl engine: FP64 geometry preprocessing, the
// C-ABI declared in include/dgmax.h, and the small support kernels (frame
// conversion, FP64 energy reduction).  The per-order phase kernels are
// generated (gen/emit.py) and compiled in their own translation units.
//
// Storage frames.  The ABI exchanges reference covariant coefficients uhat
// (physical field F^{-T} uhat, Section 3.2.1).  Inside dgm_step the state is
// kept in the frame S = det(A) A^{-T} K^{-1} uhat, where K = F^T F / (eps J) is
// the flat-element mass inverse of Section 3.3.1 (signed J carries the sign of
// the covariant curl identity) and A holds the three derivative directions.
// In that frame the mass inverse moves to the input side (w = M S with
// M = A K A^T / det A symmetric) and the update of each component is
// independent of the other two, which lets the phase kernel finish one
// component at a time.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/dgmax.h"
#include "dense.h"
#include "launch.h"
#include "generated/frame.inc"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(e_ == hipErrorOutOfMemory ? DGM_ERR_OOM : DGM_ERR_HIP,                \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                   \
  } while (0)

constexpr int64_t kMaxElements = (int64_t(1) << 28) - 64;

int num_modes(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
int num_face_modes(int p) { return (p + 1) * (p + 2) / 2; }
// Values of one field's trace buffer: whole 64-element tiles (the last one padded).
size_t trace_words(int64_t K, int p) { return (size_t)((K + 63) / 64) * 64 * trace_elem_stride(num_face_modes(p)); }
// Bytes a leapfrog step streams through (both fields and both trace buffers); above
// the 256 MB last-level cache the phase kernels use nontemporal field accesses.
constexpr size_t kStreamingBytes = size_t(256) << 20;
size_t step_bytes(int64_t K, int p, size_t rsize) {
  return (2 * (size_t)3 * num_modes(p) * (size_t)K + 2 * trace_words(K, p)) * rsize;
}

// ---------------------------------------------------------------- kernels
// X_m <- P X_m for every mode m of every element, P = (Minv A) (to the stored
// frame) or (Ainv M) (back to covariant).  M, Minv are symmetric, stored (6,K).
template <typename R>
__global__ void convert_kernel(R* __restrict__ X, const R* __restrict__ Msym, int N, int K, int to_stored,
                               double a00, double a01, double a02, double a10, double a11, double a12,
                               double a20, double a21, double a22) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K) return;
  const size_t Ks = (size_t)K;
  const double s00 = Msym[0 * Ks + e], s01 = Msym[1 * Ks + e], s02 = Msym[2 * Ks + e];
  const double s11 = Msym[3 * Ks + e], s12 = Msym[4 * Ks + e], s22 = Msym[5 * Ks + e];
  const double S[3][3] = {{s00, s01, s02}, {s01, s11, s12}, {s02, s12, s22}};
  const double C[3][3] = {{a00, a01, a02}, {a10, a11, a12}, {a20, a21, a22}};
  double P[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int q = 0; q < 3; ++q) acc += to_stored ? S[r][q] * C[q][c] : C[r][q] * S[q][c];
      P[r][c] = acc;
    }
  for (int m = 0; m < N; ++m) {
    R* x0 = X + ((size_t)(0 * N + m)) * Ks + e;
    R* x1 = X + ((size_t)(1 * N + m)) * Ks + e;
    R* x2 = X + ((size_t)(2 * N + m)) * Ks + e;
    const double v0 = *x0, v1 = *x1, v2 = *x2;
    *x0 = (R)(P[0][0] * v0 + P[0][1] * v1 + P[0][2] * v2);
    *x1 = (R)(P[1][0] * v0 + P[1][1] * v1 + P[1][2] * v2);
    *x2 = (R)(P[2][0] * v0 + P[2][1] * v1 + P[2][2] * v2);
  }
}

// Elementwise kernels over whole fields (3 N K values, which can exceed the 2^32
// work-items of one launch) loop with a grid stride over a capped grid.
constexpr int kFlatThreads = 256;
constexpr size_t kFlatMaxBlocks = 65536;
inline unsigned flat_blocks(size_t n) {
  return (unsigned)std::min<size_t>(kFlatMaxBlocks, std::max<size_t>(1, (n + kFlatThreads - 1) / kFlatThreads));
}

template <typename R>
__global__ void fill_kernel(R* __restrict__ X, size_t n, R v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) X[i] = v;
}

// Y <- X + a * Y  (used to form H_next = H + dt dH in place of dH)
template <typename R>
__global__ void xpay_kernel(R* __restrict__ Y, const R* __restrict__ X, size_t n, double a) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    Y[i] = (R)((double)X[i] + a * (double)Y[i]);
}

// Mass-weighted dot products in FP64: out[b] = sum over the block's elements of
// sum_m A_m^T G_e B_m, with G = |J| eps F^{-1} F^{-T} symmetric (6,K).
// Deterministic: fixed block partition, fixed tree, separate final pass.
constexpr int kRedThreads = 256;

template <typename R>
__global__ void __launch_bounds__(kRedThreads) mdot_partial_kernel(const R* __restrict__ A, const R* __restrict__ B,
                                                                   const double* __restrict__ G, int N, int K,
                                                                   double* __restrict__ partial) {
  __shared__ double red[kRedThreads];
  const int e = blockIdx.x * kRedThreads + threadIdx.x;
  double acc = 0.0;
  if (e < K) {
    const size_t Ks = (size_t)K;
    const double g00 = G[0 * Ks + e], g01 = G[1 * Ks + e], g02 = G[2 * Ks + e];
    const double g11 = G[3 * Ks + e], g12 = G[4 * Ks + e], g22 = G[5 * Ks + e];
    for (int m = 0; m < N; ++m) {
      const double a0 = A[(size_t)(0 * N + m) * Ks + e], a1 = A[(size_t)(1 * N + m) * Ks + e],
                   a2 = A[(size_t)(2 * N + m) * Ks + e];
      const double b0 = B[(size_t)(0 * N + m) * Ks + e], b1 = B[(size_t)(1 * N + m) * Ks + e],
                   b2 = B[(size_t)(2 * N + m) * Ks + e];
      acc += a0 * (g00 * b0 + g01 * b1 + g02 * b2) + a1 * (g01 * b0 + g11 * b1 + g12 * b2) +
             a2 * (g02 * b0 + g12 * b1 + g22 * b2);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kRedThreads) final_sum_kernel(const double* __restrict__ partial, int n,
                                                                double* __restrict__ out) {
  __shared__ double red[kRedThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kRedThreads) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// Partial sums (FP64) of the plain dot product of two arrays; one per block.
template <typename R>
__global__ void __launch_bounds__(kRedThreads) dot_partial_kernel(const R* __restrict__ A, const R* __restrict__ B,
                                                                  size_t n, double* __restrict__ partial) {
  __shared__ double red[kRedThreads];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kRedThreads)
    acc += (double)A[i] * (double)B[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Partial sums (FP64) of the face-unknown energy product sum over owner sides and face
// modes of a_m^T W b_m, with a, b the face unknowns (layout ((k NF + m) 4 + f) K + e)
// and W the side's symmetric 2x2 weight (12,K): (h_F/alpha) 2|F| G^{-1}, zero on
// sides that do not own their face.
template <typename R>
__global__ void __launch_bounds__(kRedThreads) fdot_partial_kernel(const R* __restrict__ A, const R* __restrict__ B,
                                                                   const double* __restrict__ W, int NF, int K,
                                                                   double* __restrict__ partial) {
  __shared__ double red[kRedThreads];
  const int e = blockIdx.x * kRedThreads + threadIdx.x;
  double acc = 0.0;
  if (e < K) {
    const size_t Ks = (size_t)K;
    for (int f = 0; f < 4; ++f) {
      const double w00 = W[(3 * f + 0) * Ks + e], w01 = W[(3 * f + 1) * Ks + e], w11 = W[(3 * f + 2) * Ks + e];
      if (w00 == 0.0 && w01 == 0.0 && w11 == 0.0) continue;
      for (int m = 0; m < NF; ++m) {
        const size_t i0 = ((size_t)(m * 4 + f)) * Ks + e, i1 = ((size_t)((NF + m) * 4 + f)) * Ks + e;
        const double a0 = A[i0], a1 = A[i1], b0 = B[i0], b1 = B[i1];
        acc += w00 * a0 * b0 + w01 * (a0 * b1 + a1 * b0) + w11 * a1 * b1;
      }
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// SplitMix64 (Steele, Lea, Flood 2014) mapped to [-1, 1): start vector of the
// power iteration, identical to the host reference generator.
template <typename R>
__global__ void splitmix_fill_kernel(R* __restrict__ X, size_t n, unsigned long long seed) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    unsigned long long z = seed + (unsigned long long)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    X[i] = (R)((double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0);
  }
}

// Conjugate gradients for the approximate mass matrix of a material that varies inside
// the elements (Section 3.3.2).  The scalars stay in device memory, so an iteration
// makes no host round trip: rz[0] = r.z, pt = p.t.
// x += alpha p, r -= alpha t, alpha = r.z / p.t (zero once the residual is zero)
template <typename R>
__global__ void cg_xr_kernel(R* __restrict__ x, R* __restrict__ r, const R* __restrict__ p, const R* __restrict__ t,
                             size_t n, const double* __restrict__ rz, const double* __restrict__ pt) {
  const double alpha = *pt != 0.0 ? *rz / *pt : 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    x[i] = (R)((double)x[i] + alpha * (double)p[i]);
    r[i] = (R)((double)r[i] - alpha * (double)t[i]);
  }
}

// t = mbar_e r with mbar_e the mean of the element's four vertex values (the
// approximate inverse is close to 1 / mbar_e, so this is the preconditioner; also the
// start value of the solution).  Field layout (3,N,K): element e = i mod K.
template <typename R>
__global__ void cg_precond_kernel(R* __restrict__ t, const R* __restrict__ r, const R* __restrict__ mat, size_t n,
                                  int K) {
  const size_t Ks = (size_t)K;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const size_t e = i % Ks;
    const double mbar = 0.25 * ((double)mat[e] + (double)mat[Ks + e] + (double)mat[2 * Ks + e] + (double)mat[3 * Ks + e]);
    t[i] = (R)(mbar * (double)r[i]);
  }
}

// p = t + beta p, beta = rz_new / rz_old
template <typename R>
__global__ void cg_p_kernel(R* __restrict__ p, const R* __restrict__ t, size_t n, const double* __restrict__ rz_new,
                            const double* __restrict__ rz_old) {
  const double beta = *rz_old != 0.0 ? *rz_new / *rz_old : 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = (R)((double)t[i] + beta * (double)p[i]);
}

template <typename A, typename B>
__global__ void cast_kernel(B* __restrict__ out, const A* __restrict__ in, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = (B)in[i];
}

template <typename R>
__global__ void scale_kernel(R* __restrict__ X, size_t n, const double* __restrict__ d) {
  const double r = sqrt(*d);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    X[i] = (R)(-(double)X[i] / r);
}

}  // namespace

// ---------------------------------------------------------------- mesh
struct dgm_mesh {
  int64_t K = 0;
  int p = 0;    // order of H (the mesh's order); E has order pE = p or p + 1 (mixed orders)
  int pE = 0;
  std::vector<double> F;   // (K,9) row-major 3x3, columns v1-v0, v2-v0, v3-v0 (sorted vertices)
  std::vector<double> J;   // signed det F
  std::vector<int> nbr;    // (4,K)
  std::vector<unsigned char> perm;  // (K,4): caller's position of each sorted vertex
  // device: one block (d_geom) holds the neighbour codes and every per-element factor;
  // the pointers below point into it and are never freed on their own
  void* d_geom = nullptr;
  size_t geom_off[12] = {};                  // byte offsets of the arrays, see geom_layout
  int* d_nbr = nullptr;
  float* d_M32[2] = {nullptr, nullptr};      // E, H: w = M S
  double* d_M64[2] = {nullptr, nullptr};
  float* d_Minv32[2] = {nullptr, nullptr};   // S = Minv A uhat
  double* d_Minv64[2] = {nullptr, nullptr};
  double* d_G[2] = {nullptr, nullptr};       // |J| eps F^-1 F^-T (energy)
  void* d_scratch = nullptr;
  size_t scratch_bytes = 0;
  void* d_T = nullptr;      // element-major traces of E then H (K x ES each)
  size_t T_bytes = 0;
  double* d_partial = nullptr;
  int partial_n = 0;
  double* d_res = nullptr;  // four FP64 reduction results (energies)
  int64_t check_every = 0;  // dgm_step: steps between finiteness checks (0: none)
  // stabilised flux (Section 2.1): alpha = stab_alpha0 p^2 once dgm_set_stab_alpha was
  // called; per owner side of every face the FP32/FP64 2x2 update matrices (16,K) and
  // the FP64 energy weights (12,K), built for order stab_p in one device block
  double stab_alpha0 = 0.0;
  int stab_p = 0;
  void* d_stab = nullptr;
  float* d_SC32 = nullptr;
  double* d_SC64 = nullptr;
  double* d_WF = nullptr;
  // material linear on every element (dgm_set_material_linear): the mass inverse is the
  // approximate one of Section 3.3.2, the metrics above are those of unit material, and
  // d_var holds eps then mu at the sorted vertices, (4,K) each, in FP32 then FP64
  bool varmat = false;
  void* d_var = nullptr;
  float* d_var32[2] = {nullptr, nullptr};
  double* d_var64[2] = {nullptr, nullptr};
  // dense matrix-core variant: operators per precision (BF16, FP16) and jump scratch
  DenseOps* dense[2] = {nullptr, nullptr};
  float* d_jump = nullptr;
  size_t jump_floats = 0;
};

namespace {

// Order of field fld (0: E, 1: H); they differ only with mixed orders (dgm_set_orders).
int ford(const dgm_mesh* m, int fld) { return fld == 0 ? m->pE : m->p; }
bool mixed(const dgm_mesh* m) { return m->pE != m->p; }
size_t field_len(const dgm_mesh* m, int fld) { return (size_t)3 * num_modes(ford(m, fld)) * (size_t)m->K; }
size_t mesh_step_bytes(const dgm_mesh* m, size_t rsize) {
  return (field_len(m, 0) + field_len(m, 1) + trace_words(m->K, m->pE) + trace_words(m->K, m->p)) * rsize;
}

int ensure_scratch(dgm_mesh* m, size_t bytes) {
  if (m->scratch_bytes >= bytes) return DGM_OK;
  if (m->d_scratch) HIP_TRY(hipFree(m->d_scratch));
  m->d_scratch = nullptr;
  m->scratch_bytes = 0;
  HIP_TRY(hipMalloc(&m->d_scratch, bytes));
  m->scratch_bytes = bytes;
  return DGM_OK;
}

// Trace buffers of both fields (E, then H) in precision R, grown on demand.
template <typename R>
int ensure_traces(dgm_mesh* m, R** TE, R** TH) {
  const size_t per = trace_words(m->K, m->pE);
  const size_t bytes = (per + trace_words(m->K, m->p)) * sizeof(R);
  if (m->T_bytes < bytes) {
    if (m->d_T) HIP_TRY(hipFree(m->d_T));
    m->d_T = nullptr;
    m->T_bytes = 0;
    HIP_TRY(hipMalloc(&m->d_T, bytes));
    m->T_bytes = bytes;
  }
  *TE = static_cast<R*>(m->d_T);
  *TH = *TE + per;
  return DGM_OK;
}

void sym6(const double S[3][3], double* out6) {
  out6[0] = S[0][0]; out6[1] = S[0][1]; out6[2] = S[0][2];
  out6[3] = S[1][1]; out6[4] = S[1][2]; out6[5] = S[2][2];
}

bool inv3(const double a[3][3], double r[3][3]) {
  const double det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                     a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                     a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
  if (det == 0.0 || !std::isfinite(det)) return false;
  r[0][0] = (a[1][1] * a[2][2] - a[1][2] * a[2][1]) / det;
  r[0][1] = (a[0][2] * a[2][1] - a[0][1] * a[2][2]) / det;
  r[0][2] = (a[0][1] * a[1][2] - a[0][2] * a[1][1]) / det;
  r[1][0] = (a[1][2] * a[2][0] - a[1][0] * a[2][2]) / det;
  r[1][1] = (a[0][0] * a[2][2] - a[0][2] * a[2][0]) / det;
  r[1][2] = (a[0][2] * a[1][0] - a[0][0] * a[1][2]) / det;
  r[2][0] = (a[1][0] * a[2][1] - a[1][1] * a[2][0]) / det;
  r[2][1] = (a[0][1] * a[2][0] - a[0][0] * a[2][1]) / det;
  r[2][2] = (a[0][0] * a[1][1] - a[0][1] * a[1][0]) / det;
  return true;
}

// Arrays of the per-mesh device block, in order; the material-dependent ones follow the
// neighbour codes contiguously so that one copy uploads them.  A device allocation costs
// about as much as a small mesh's whole set-up, hence one block instead of eleven.
enum GeomArray { kNbr, kM32E, kM32H, kMinv32E, kMinv32H, kM64E, kM64H, kMinv64E, kMinv64H, kGE, kGH, kGeomArrays };
static_assert(sizeof(dgm_mesh::geom_off) == (kGeomArrays + 1) * sizeof(size_t), "one offset per array plus the total");

// Byte offsets (256-byte aligned) of the arrays for K elements; off[kGeomArrays] = total.
void geom_layout(int64_t K, size_t off[kGeomArrays + 1]) {
  const size_t k6 = 6 * (size_t)K;
  const size_t sz[kGeomArrays] = {4 * (size_t)K * sizeof(int), k6 * sizeof(float), k6 * sizeof(float),
                                  k6 * sizeof(float), k6 * sizeof(float), k6 * sizeof(double), k6 * sizeof(double),
                                  k6 * sizeof(double), k6 * sizeof(double), k6 * sizeof(double), k6 * sizeof(double)};
  size_t o = 0;
  for (int i = 0; i < kGeomArrays; ++i) {
    off[i] = o;
    o += (sz[i] + 255) & ~size_t(255);
  }
  off[kGeomArrays] = o;
}


int material_impl(dgm_mesh* m, const double* eps, const double* mu) {
  const int64_t K = m->K;
  const double(*A)[3] = reinterpret_cast<const double(*)[3]>(kFrameA);
  // host image of the material part of the device block: every value is checked and
  // computed before the one upload, so a rejected material leaves the mesh unchanged
  const size_t* off = m->geom_off;
  std::vector<unsigned char> img(off[kGeomArrays] - off[kM32E]);
  const auto at = [&](int arr) { return img.data() + (off[arr] - off[kM32E]); };
  for (int arr = kM32E; arr < kGeomArrays; ++arr) {  // zero the alignment padding
    const size_t used = 6 * (size_t)K * (arr < kM64E ? sizeof(float) : sizeof(double));
    std::memset(at(arr) + used, 0, off[arr + 1] - off[arr] - used);
  }
  for (int fld = 0; fld < 2; ++fld) {
    const double* mat = fld == 0 ? eps : mu;
    float* M32 = reinterpret_cast<float*>(at(kM32E + fld));
    float* Minv32 = reinterpret_cast<float*>(at(kMinv32E + fld));
    double* M64 = reinterpret_cast<double*>(at(kM64E + fld));
    double* Minv64 = reinterpret_cast<double*>(at(kMinv64E + fld));
    double* G = reinterpret_cast<double*>(at(kGE + fld));
    for (int64_t e = 0; e < K; ++e) {
      const double c = mat ? mat[e] : 1.0;
      if (!(c > 0.0) || !std::isfinite(c))
        return fail(DGM_ERR_MATERIAL, "material value must be finite and > 0 (element " + std::to_string(e) + ")");
      double Fm[3][3], FtF[3][3], Fi[3][3], FiFiT[3][3], Km[3][3], AK[3][3], Mm[3][3], Mi[3][3];
      std::memcpy(Fm, &m->F[9 * e], sizeof(Fm));
      const double Je = m->J[e];
      for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) {
          double acc = 0.0;
          for (int q = 0; q < 3; ++q) acc += Fm[q][r] * Fm[q][s];
          FtF[r][s] = acc;
          Km[r][s] = acc / (c * Je);  // flat-element mass inverse, sign of J included
        }
      inv3(Fm, Fi);
      for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) {
          double acc = 0.0;
          for (int q = 0; q < 3; ++q) acc += Fi[r][q] * Fi[s][q];
          FiFiT[r][s] = std::fabs(Je) * c * acc;
        }
      for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) {
          double acc = 0.0;
          for (int q = 0; q < 3; ++q) acc += A[r][q] * Km[q][s];
          AK[r][s] = acc;
        }
      for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) {
          double acc = 0.0;
          for (int q = 0; q < 3; ++q) acc += AK[r][q] * A[s][q];
          Mm[r][s] = acc / kFrameDetA;
        }
      // symmetrise against rounding before inverting
      for (int r = 0; r < 3; ++r)
        for (int s = r + 1; s < 3; ++s) Mm[r][s] = Mm[s][r] = 0.5 * (Mm[r][s] + Mm[s][r]);
      if (!inv3(Mm, Mi)) return fail(DGM_ERR_MESH_DEGENERATE, "singular element metric");
      double o6[6];
      sym6(Mm, o6);
      for (int q = 0; q < 6; ++q) M64[q * K + e] = o6[q], M32[q * K + e] = (float)o6[q];
      sym6(Mi, o6);
      for (int q = 0; q < 6; ++q) Minv64[q * K + e] = o6[q], Minv32[q * K + e] = (float)o6[q];
      sym6(FiFiT, o6);
      for (int q = 0; q < 6; ++q) G[q * K + e] = o6[q];
      (void)FtF;
    }
  }
  HIP_TRY(hipMemcpy(static_cast<unsigned char*>(m->d_geom) + off[kM32E], img.data(), img.size(),
                    hipMemcpyHostToDevice));
  return DGM_OK;
}

template <typename R> R* Mdev(dgm_mesh* m, int fld);
template <> float* Mdev<float>(dgm_mesh* m, int fld) { return m->d_M32[fld]; }
template <> double* Mdev<double>(dgm_mesh* m, int fld) { return m->d_M64[fld]; }
template <typename R> R* Minvdev(dgm_mesh* m, int fld);
template <> float* Minvdev<float>(dgm_mesh* m, int fld) { return m->d_Minv32[fld]; }
template <> double* Minvdev<double>(dgm_mesh* m, int fld) { return m->d_Minv64[fld]; }

hipError_t phase(const PhaseArgs<float>& a, int p) { return kPhaseF32[p](a); }
hipError_t phase(const PhaseArgs<double>& a, int p) { return kPhaseF64[p](a); }
hipError_t mix(const PhaseArgs<float>& a, int p, int dir) { return kMixF32[p](a, dir); }
hipError_t mix(const PhaseArgs<double>& a, int p, int dir) { return kMixF64[p](a, dir); }
hipError_t trace(const TraceArgs<float>& a, int p) { return kTraceF32[p](a); }
hipError_t trace(const TraceArgs<double>& a, int p) { return kTraceF64[p](a); }
template <typename R> bool mass_built(int p);
template <> bool mass_built<float>(int p) { return p >= 1 && p <= DGM_MAX_ORDER_F32 && kMassF32[p] != nullptr; }
template <> bool mass_built<double>(int p) { return p >= 1 && p <= DGM_MAX_ORDER_F64 && kMassF64[p] != nullptr; }
hipError_t mass(const MassArgs<float>& a, int p) { return kMassF32[p](a); }
hipError_t mass(const MassArgs<double>& a, int p) { return kMassF64[p](a); }
template <typename R> const R* vardev(const dgm_mesh* m, int fld);
template <> const float* vardev<float>(const dgm_mesh* m, int fld) { return m->d_var32[fld]; }
template <> const double* vardev<double>(const dgm_mesh* m, int fld) { return m->d_var64[fld]; }

// Whether the kernels of order p are built for dtype.  The launcher tables are
// indexed by order and hold nullptr for orders that were not generated.
bool order_built(int p, int dtype) {
  if (p < 1 || p > DGM_MAX_ORDER_F32) return false;
  if (dtype == DGM_F32) return kPhaseF32[p] != nullptr && kTraceF32[p] != nullptr && kBatchF32[p] != nullptr;
  return p <= DGM_MAX_ORDER_F64 && kPhaseF64[p] != nullptr && kTraceF64[p] != nullptr;
}

// Mixed orders (H of order p, E of order p + 1): the pair's phase kernels and both orders'
// trace kernels must be built for dtype.
bool mixed_built(int p, int dtype) {
  if (p < 1 || p + 1 > DGM_MAX_ORDER_F32) return false;
  if (dtype == DGM_F32) return kMixF32[p] != nullptr && kTraceF32[p] != nullptr && kTraceF32[p + 1] != nullptr;
  return p + 1 <= DGM_MAX_ORDER_F64 && kMixF64[p] != nullptr && kTraceF64[p] != nullptr && kTraceF64[p + 1] != nullptr;
}

int check_order(dgm_mesh* m, int dtype) {
  if (!m) return fail(DGM_ERR_ARG, "null mesh");
  if (dtype != DGM_F32 && dtype != DGM_F64) return fail(DGM_ERR_ARG, "dtype must be DGM_F32 or DGM_F64");
  if (m->p < 1) return fail(DGM_ERR_STATE, "order not set (dgm_set_order)");
  if (m->varmat && !(dtype == DGM_F32 ? mass_built<float>(m->pE) && mass_built<float>(m->p)
                                      : mass_built<double>(m->pE) && mass_built<double>(m->p)))
    return fail(DGM_ERR_ARG, "mass kernels of the orders not compiled for this dtype");
  if (mixed(m)) {
    if (!mixed_built(m->p, dtype))
      return fail(DGM_ERR_ARG, "mixed orders (" + std::to_string(m->pE) + ", " + std::to_string(m->p) +
                                   ") not compiled for this dtype");
    return DGM_OK;
  }
  if (!order_built(m->p, dtype))
    return fail(DGM_ERR_ARG, "order " + std::to_string(m->p) + " not compiled for this dtype (max " +
                                 std::to_string(dtype == DGM_F32 ? DGM_MAX_ORDER_F32 : DGM_MAX_ORDER_F64) + ")");
  return DGM_OK;
}

int check_equal_orders(const dgm_mesh* m, const char* what) {
  if (mixed(m)) return fail(DGM_ERR_STATE, std::string(what) + " needs equal orders for E and H");
  return DGM_OK;
}

// Paths built for piecewise-constant material only (not for dgm_set_material_linear).
int check_constant_material(const dgm_mesh* m, const char* what) {
  if (m->varmat) return fail(DGM_ERR_STATE, std::string(what) + " needs piecewise-constant material (dgm_set_material)");
  return DGM_OK;
}

template <typename R>
int convert(dgm_mesh* m, R* X, int fld, bool to_stored, hipStream_t s) {
  const double* C = to_stored ? kFrameA : kFrameAinv;
  const R* Msym = to_stored ? Minvdev<R>(m, fld) : Mdev<R>(m, fld);
  const int threads = 256;
  hipLaunchKernelGGL(convert_kernel<R>, dim3((unsigned)((m->K + threads - 1) / threads)), dim3(threads), 0, s, X, Msym,
                     num_modes(ford(m, fld)), (int)m->K, to_stored ? 1 : 0, C[0], C[1], C[2], C[3], C[4], C[5], C[6], C[7],
                     C[8]);
  HIP_TRY(hipGetLastError());
  return DGM_OK;
}

template <typename R>
int fill(R* X, size_t n, R v, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel<R>, dim3(flat_blocks(n)), dim3(kFlatThreads), 0, s, X, n, v);
  HIP_TRY(hipGetLastError());
  return DGM_OK;
}

// Element-major traces T of the stored-frame field U (fld 0: E, 1: H).
template <typename R>
int run_trace(dgm_mesh* m, const R* U, int fld, R* T, hipStream_t s) {
  TraceArgs<R> a;
  a.U = U;
  a.MU = Mdev<R>(m, fld);
  a.nbr = m->d_nbr;
  a.T = T;
  a.K = (int)m->K;
  a.blocks = (int)((m->K + 63) / 64);
  a.stream = s;
  HIP_TRY(trace(a, ford(m, fld)));
  return DGM_OK;
}

// Approximate mass inverse of field fld (material linear on the elements):
// V = (acc ? V : 0) + s P X, component by component (X, V in any one frame).
template <typename R>
int run_mass(dgm_mesh* m, const R* X, R* V, int fld, double sc, bool acc, hipStream_t s) {
  const int p = ford(m, fld);
  if (!mass_built<R>(p)) return fail(DGM_ERR_ARG, "mass kernel of order " + std::to_string(p) + " not built for this dtype");
  MassArgs<R> a;
  a.X = X;
  a.V = V;
  a.mat = vardev<R>(m, fld);
  a.s = (R)sc;
  a.acc = acc ? 1 : 0;
  a.K = (int)m->K;
  a.blocks = (int)((m->K + 63) / 64);
  a.stream = s;
  HIP_TRY(mass(a, p));
  return DGM_OK;
}

// One phase on stored-frame data.  fld_u: 0 if U is E (H update), 1 if U is H.
// Tin holds the traces of U; Tout (or nullptr) receives those of the updated V.
template <typename R>
const R* SCdev(const dgm_mesh* m);
template <>
const float* SCdev<float>(const dgm_mesh* m) { return m->d_SC32; }
template <>
const double* SCdev<double>(const dgm_mesh* m) { return m->d_SC64; }

// With HF (stabilised flux): the H phase (fld_u 0) advances the face unknowns by fdt
// times their rate; the E phase reads them.
// overwrite: V = sdt * rate without reading V (central flux, equal orders only; the
// callers check that).
template <typename R>
int run_phase(dgm_mesh* m, const R* U, R* V, int fld_u, double sdt, const R* Tin, R* Tout, hipStream_t s,
              R* HF = nullptr, double fdt = 0.0, bool overwrite = false) {
  PhaseArgs<R> a;
  a.U = U;
  a.V = V;
  a.MU = Mdev<R>(m, fld_u);
  a.MV = Mdev<R>(m, 1 - fld_u);
  a.nbr = m->d_nbr;
  a.Tin = Tin;
  a.Tout = Tout;
  a.sdt = (R)sdt;
  a.wall = fld_u == 0 ? (R)-1 : (R)1;
  a.K = (int)m->K;
  a.blocks = (int)((m->K + 63) / 64);
  a.streaming = mesh_step_bytes(m, sizeof(R)) > kStreamingBytes;
  a.stream = s;
  a.HF = HF;
  a.SC = HF ? SCdev<R>(m) : nullptr;
  a.fdt = (R)fdt;
  a.overwrite = overwrite ? 1 : 0;
  if (overwrite && (HF || mixed(m) || Tout)) return fail(DGM_ERR_STATE, "rate-only phase needs the central flux and equal orders");
  if (mixed(m)) {
    if (HF) return fail(DGM_ERR_STATE, "the stabilised flux needs equal orders");
    HIP_TRY(mix(a, m->p, fld_u));
  } else {
    HIP_TRY(phase(a, m->p));
  }
  return DGM_OK;
}

// Covariant rate: out = d/dt of the other field from the covariant input `in`.
// fld_u = 0: in = E, out = dH;  fld_u = 1: in = H, out = dE.
// With a material linear on the elements (m->varmat) the metrics are those of unit
// material and the approximate mass inverse follows (with_mass; without it the rate is
// the unit-material one, which the dt estimate needs); the scratch then holds the
// stored-frame copy of the input and the unit-material rate.
template <typename R>
int rate_impl(dgm_mesh* m, const R* in, R* out, int fld_u, hipStream_t s, R* HF = nullptr, double fdt = 0.0,
              bool with_mass = true) {
  const size_t n = field_len(m, fld_u), n_out = field_len(m, 1 - fld_u);
  const bool var = m->varmat && with_mass;
  int rc;
  if ((rc = ensure_scratch(m, (n + (var ? n_out : 0)) * sizeof(R)))) return rc;
  R* tmp = static_cast<R*>(m->d_scratch);
  R* dst = var ? tmp + n : out;
  R* T[2];
  if ((rc = ensure_traces<R>(m, &T[0], &T[1]))) return rc;
  HIP_TRY(hipMemcpyAsync(tmp, in, n * sizeof(R), hipMemcpyDeviceToDevice, s));
  if ((rc = convert<R>(m, tmp, fld_u, true, s))) return rc;
  if ((rc = run_trace<R>(m, tmp, fld_u, T[fld_u], s))) return rc;
  // the phase writes the rate into dst directly where it can, else adds it to zeros
  const bool direct = !HF && !mixed(m);
  if (!direct && (rc = fill<R>(dst, n_out, (R)0, s))) return rc;
  if ((rc = run_phase<R>(m, tmp, dst, fld_u, fld_u == 0 ? -1.0 : 1.0, T[fld_u], nullptr, s, HF, fdt, direct))) return rc;
  if (var && (rc = run_mass<R>(m, dst, out, 1 - fld_u, 1.0, false, s))) return rc;
  return convert<R>(m, out, 1 - fld_u, false, s);
}

constexpr int kDotBlocks = 512;

int ensure_partial(dgm_mesh* m, int nb) {
  if (m->partial_n >= nb) return DGM_OK;
  if (m->d_partial) HIP_TRY(hipFree(m->d_partial));
  m->d_partial = nullptr;
  m->partial_n = 0;
  HIP_TRY(hipMalloc(&m->d_partial, nb * sizeof(double)));
  m->partial_n = nb;
  return DGM_OK;
}

// FP64 sum of squares of both fields (any frame), synchronised: finite iff every
// coefficient is finite (short of overflow in the squares).
// Device workspace of a run of leapfrog steps: the two trace buffers, kDotBlocks FP64
// partial sums and two FP64 results (the last two only for checks and probes).
template <typename R>
struct StepWork {
  R* TE = nullptr;
  R* TH = nullptr;
  R* rate = nullptr;  // unit-material rate of the updated field (material linear on the elements)
  double* partial = nullptr;
  double* res = nullptr;
};

// FP64 sum of squares of both fields (any frame), synchronised: finite iff every
// coefficient is finite (short of overflow in the squares).
template <typename R>
int finite_state(const StepWork<R>& ws, const R* E, const R* H, size_t nE, size_t nH, int nb, bool* ok,
                 hipStream_t s) {
  for (int f = 0; f < 2; ++f) {
    const R* X = f == 0 ? E : H;
    hipLaunchKernelGGL(dot_partial_kernel<R>, dim3(nb), dim3(kRedThreads), 0, s, X, X, f == 0 ? nE : nH, ws.partial);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(kRedThreads), 0, s, ws.partial, nb, ws.res + f);
    HIP_TRY(hipGetLastError());
  }
  double h[2];
  HIP_TRY(hipMemcpyAsync(h, ws.res, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *ok = std::isfinite(h[0]) && std::isfinite(h[1]);
  return DGM_OK;
}

// Workspace of dgm_step / dgm_step_probe, owned by the mesh handle (grown on demand).
template <typename R>
int mesh_work(dgm_mesh* m, bool reductions, StepWork<R>* ws) {
  int rc;
  if ((rc = ensure_traces<R>(m, &ws->TE, &ws->TH))) return rc;
  if (m->varmat) {
    if ((rc = ensure_scratch(m, std::max(field_len(m, 0), field_len(m, 1)) * sizeof(R)))) return rc;
    ws->rate = static_cast<R*>(m->d_scratch);
  }
  if (reductions) {
    if ((rc = ensure_partial(m, kDotBlocks))) return rc;
    if (!m->d_res) HIP_TRY(hipMalloc(&m->d_res, 4 * sizeof(double)));
    ws->partial = m->d_partial;
    ws->res = m->d_res;
  }
  return DGM_OK;
}

// With w and d_sig: after step n, d_sig[n] = sum_i w_i E_i (E in the stored frame).
// With m->check_every > 0 the state is checked after every check_every steps (and after
// the last); a non-finite state ends the run (fields converted back) with DGM_ERR_UNSTABLE.
// ws: trace buffers (always) and, for checks or probes, the reduction buffers.
template <typename R>
int step_impl(dgm_mesh* m, R* E, R* H, double dt, int64_t nsteps, hipStream_t s, const StepWork<R>& ws,
              const R* w = nullptr, double* d_sig = nullptr, R* HF = nullptr) {
  int rc;
  if (nsteps == 0) return DGM_OK;
  const size_t n = field_len(m, 0), nH = field_len(m, 1);
  const int nb = (int)std::min<size_t>(kDotBlocks, (std::max(n, nH) + kRedThreads - 1) / kRedThreads);
  const int64_t every = m->check_every;
  R* const TE = ws.TE;
  R* const TH = ws.TH;
  if ((rc = convert<R>(m, E, 0, true, s))) return rc;
  if ((rc = convert<R>(m, H, 1, true, s))) return rc;
  if ((rc = run_trace<R>(m, E, 0, TE, s))) return rc;
  for (int64_t it = 0; it < nsteps; ++it) {
    // H update from curl E (writes the traces of H), then E update from curl H
    // (writes the traces of E for the next step, except after the last one)
    if (m->varmat) {
      // unit-material rate, then its approximate mass inverse into the field, then
      // the traces of the updated field
      const bool direct = !mixed(m);
      if (!direct && (rc = fill<R>(ws.rate, nH, (R)0, s))) return rc;
      if ((rc = run_phase<R>(m, E, ws.rate, 0, -1.0, TE, nullptr, s, nullptr, 0.0, direct))) return rc;
      if ((rc = run_mass<R>(m, ws.rate, H, 1, dt, true, s))) return rc;
      if ((rc = run_trace<R>(m, H, 1, TH, s))) return rc;
      if (!direct && (rc = fill<R>(ws.rate, n, (R)0, s))) return rc;
      if ((rc = run_phase<R>(m, H, ws.rate, 1, 1.0, TH, nullptr, s, nullptr, 0.0, direct))) return rc;
      if ((rc = run_mass<R>(m, ws.rate, E, 0, dt, true, s))) return rc;
      if (it + 1 < nsteps && (rc = run_trace<R>(m, E, 0, TE, s))) return rc;
    } else {
      if ((rc = run_phase<R>(m, E, H, 0, -dt, TE, TH, s, HF, dt))) return rc;
      if ((rc = run_phase<R>(m, H, E, 1, dt, TH, it + 1 < nsteps ? TE : nullptr, s, HF))) return rc;
    }
    if (w) {
      hipLaunchKernelGGL(dot_partial_kernel<R>, dim3(nb), dim3(kRedThreads), 0, s, (const R*)E, w, n, ws.partial);
      HIP_TRY(hipGetLastError());
      hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(kRedThreads), 0, s, ws.partial, nb, d_sig + it);
      HIP_TRY(hipGetLastError());
    }
    if (every > 0 && ((it + 1) % every == 0 || it + 1 == nsteps)) {
      bool ok = true;
      if ((rc = finite_state<R>(ws, E, H, n, nH, nb, &ok, s))) return rc;
      if (!ok) {
        if ((rc = convert<R>(m, E, 0, false, s))) return rc;
        if ((rc = convert<R>(m, H, 1, false, s))) return rc;
        return fail(DGM_ERR_UNSTABLE, "non-finite state after step " + std::to_string(it + 1) +
                                          " (time step above the stability bound?)");
      }
    }
  }
  if ((rc = convert<R>(m, E, 0, false, s))) return rc;
  return convert<R>(m, H, 1, false, s);
}

template <typename R>
int mdot(dgm_mesh* m, const R* A, const R* B, int fld, double* d_out, hipStream_t s) {
  const int nb = (int)((m->K + kRedThreads - 1) / kRedThreads);
  int rc;
  if ((rc = ensure_partial(m, nb))) return rc;
  hipLaunchKernelGGL(mdot_partial_kernel<R>, dim3(nb), dim3(kRedThreads), 0, s, A, B, m->d_G[fld], num_modes(ford(m, fld)),
                     (int)m->K, m->d_partial);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(kRedThreads), 0, s, m->d_partial, nb, d_out);
  HIP_TRY(hipGetLastError());
  return DGM_OK;
}

template <typename R>
int energy_impl(dgm_mesh* m, const R* E, const R* H, const R* Hn, double dt, double out[2], hipStream_t s) {
  const size_t n = field_len(m, 1), nE = field_len(m, 0);
  int rc;
  if (!m->d_res) HIP_TRY(hipMalloc(&m->d_res, 4 * sizeof(double)));
  double* d_res = m->d_res;
  const R* Hq = Hn;
  R* hn_buf = nullptr;
  if (!Hq) {
    // H_next = H + dt dH(E); the rate uses the first half of the scratch, H_next the second
    if ((rc = ensure_scratch(m, (nE + n) * sizeof(R)))) return rc;
    hn_buf = static_cast<R*>(m->d_scratch) + nE;
    if ((rc = rate_impl<R>(m, E, hn_buf, 0, s))) return rc;
    hipLaunchKernelGGL(xpay_kernel<R>, dim3(flat_blocks(n)), dim3(kFlatThreads), 0, s, hn_buf, H, n, dt);
    HIP_TRY(hipGetLastError());
    Hq = hn_buf;
  }
  if ((rc = mdot<R>(m, E, E, 0, d_res + 0, s))) return rc;
  if ((rc = mdot<R>(m, H, H, 1, d_res + 1, s))) return rc;
  if ((rc = mdot<R>(m, H, Hq, 1, d_res + 2, s))) return rc;
  double h[4];
  HIP_TRY(hipMemcpyAsync(h, d_res, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  out[0] = 0.5 * h[0] + 0.5 * h[1];
  out[1] = 0.5 * h[0] + 0.5 * h[2];
  if (!std::isfinite(out[0]) || !std::isfinite(out[1])) return fail(DGM_ERR_UNSTABLE, "non-finite energy");
  return DGM_OK;
}

// Solves P x = b for field fld (P the approximate mass inverse, symmetric positive
// definite per element and component) by conjugate gradients preconditioned with the
// element's mean material; x starts at that preconditioner applied to b.  r, p, t are
// work vectors of b's length, d four FP64 device scalars.  Stops once r.z has fallen
// by tol^2 (checked on the host every 8 iterations) or after 400 iterations.
template <typename T>
int mass_solve(dgm_mesh* m, int fld, const T* b, T* x, T* r, T* p, T* t, double* d, double tol, hipStream_t s) {
  const size_t n = field_len(m, fld);
  const unsigned fb = flat_blocks(n);
  const int nb = (int)std::min<size_t>(kDotBlocks, (n + kRedThreads - 1) / kRedThreads);
  const T* mat = vardev<T>(m, fld);
  int rc;
  if ((rc = ensure_partial(m, nb))) return rc;
  auto dot = [&](const T* A, const T* B, double* out) -> int {
    hipLaunchKernelGGL(dot_partial_kernel<T>, dim3(nb), dim3(kRedThreads), 0, s, A, B, n, m->d_partial);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(kRedThreads), 0, s, m->d_partial, nb, out);
    HIP_TRY(hipGetLastError());
    return DGM_OK;
  };
  // x = M b, r = b - P x, t = M r, p = t, d[0] = r.t, d[3] = b.M b
  hipLaunchKernelGGL(cg_precond_kernel<T>, dim3(fb), dim3(kFlatThreads), 0, s, x, b, mat, n, (int)m->K);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(r, b, n * sizeof(T), hipMemcpyDeviceToDevice, s));
  if ((rc = run_mass<T>(m, x, r, fld, -1.0, true, s))) return rc;
  hipLaunchKernelGGL(cg_precond_kernel<T>, dim3(fb), dim3(kFlatThreads), 0, s, t, b, mat, n, (int)m->K);
  HIP_TRY(hipGetLastError());
  if ((rc = dot(b, t, d + 3))) return rc;
  hipLaunchKernelGGL(cg_precond_kernel<T>, dim3(fb), dim3(kFlatThreads), 0, s, t, r, mat, n, (int)m->K);
  HIP_TRY(hipGetLastError());
  if ((rc = dot(r, t, d + 0))) return rc;
  HIP_TRY(hipMemcpyAsync(p, t, n * sizeof(T), hipMemcpyDeviceToDevice, s));
  int cur = 0;
  for (int it = 1; it <= 400; ++it) {
    if ((rc = run_mass<T>(m, p, t, fld, 1.0, false, s))) return rc;
    if ((rc = dot(p, t, d + 1))) return rc;
    hipLaunchKernelGGL(cg_xr_kernel<T>, dim3(fb), dim3(kFlatThreads), 0, s, x, r, (const T*)p, (const T*)t, n,
                       (const double*)(d + cur), (const double*)(d + 1));
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(cg_precond_kernel<T>, dim3(fb), dim3(kFlatThreads), 0, s, t, r, mat, n, (int)m->K);
    HIP_TRY(hipGetLastError());
    const int nxt = 2 - cur;  // r.z alternates between d[0] and d[2]
    if ((rc = dot(r, t, d + nxt))) return rc;
    hipLaunchKernelGGL(cg_p_kernel<T>, dim3(fb), dim3(kFlatThreads), 0, s, p, (const T*)t, n, (const double*)(d + nxt),
                       (const double*)(d + cur));
    HIP_TRY(hipGetLastError());
    cur = nxt;
    if (it % 8 == 0) {
      double h[4];
      HIP_TRY(hipMemcpyAsync(h, d, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (!std::isfinite(h[cur])) return fail(DGM_ERR_UNSTABLE, "non-finite residual in the mass solve");
      if (h[cur] <= tol * tol * h[3]) return DGM_OK;
    }
  }
  return fail(DGM_ERR_UNSTABLE, "mass solve did not converge in 400 iterations");
}

// W and Q with the approximate mass matrices (material linear on the elements).  With
// M~ = P^{-1} per component and G the unit-material metric of the covariant inner
// product, (a, M~ b) = (P^{-1} a)^T G b, so each energy needs one solve per field:
// y = P^{-1} E, z = P^{-1} H, then W = 1/2 (y, G E) + 1/2 (z, G H) and Q has H_next in
// place of H in the second term.  The solves and products run in FP64 whenever the
// FP64 kernels of both orders are built (for FP32 fields after a copy to FP64).
template <typename T, typename R>
int energy_var_core(dgm_mesh* m, const R* E, const R* H, const R* Hq, double out[2], hipStream_t s) {
  const size_t nE = field_len(m, 0), nH = field_len(m, 1), nmax = std::max(nE, nH);
  const bool cast = !std::is_same<T, R>::value;
  const size_t words = 5 * nmax + (cast ? nE + 2 * nH : 0);
  T* w = nullptr;
  HIP_TRY(hipMallocAsync(reinterpret_cast<void**>(&w), words * sizeof(T) + 5 * sizeof(double), s));
  T *y = w, *z = y + nmax, *r = z + nmax, *p = r + nmax, *t = p + nmax;
  const T *Et = reinterpret_cast<const T*>(E), *Ht = reinterpret_cast<const T*>(H), *Hqt = reinterpret_cast<const T*>(Hq);
  int rc = DGM_OK;
  if (cast) {
    T* c = t + nmax;
    hipLaunchKernelGGL((cast_kernel<R, T>), dim3(flat_blocks(nE)), dim3(kFlatThreads), 0, s, c, E, nE);
    hipLaunchKernelGGL((cast_kernel<R, T>), dim3(flat_blocks(nH)), dim3(kFlatThreads), 0, s, c + nE, H, nH);
    hipLaunchKernelGGL((cast_kernel<R, T>), dim3(flat_blocks(nH)), dim3(kFlatThreads), 0, s, c + nE + nH, Hq, nH);
    if (hipGetLastError() != hipSuccess) rc = fail(DGM_ERR_HIP, "cast kernel launch failed");
    Et = c;
    Ht = c + nE;
    Hqt = c + nE + nH;
  }
  // four FP64 scalars after the vectors, aligned to 8 bytes
  double* d = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(t + nmax + (cast ? nE + 2 * nH : 0)) + 7) &
                                        ~uintptr_t(7));
  const double tol = sizeof(T) == 8 ? 1e-13 : 1e-6;
  if (!rc) rc = mass_solve<T>(m, 0, Et, y, r, p, t, d, tol, s);
  if (!rc) rc = mass_solve<T>(m, 1, Ht, z, r, p, t, d, tol, s);
  if (!rc) rc = mdot<T>(m, y, Et, 0, m->d_res + 0, s);
  if (!rc) rc = mdot<T>(m, z, Ht, 1, m->d_res + 1, s);
  if (!rc) rc = mdot<T>(m, z, Hqt, 1, m->d_res + 2, s);
  double h[3] = {0, 0, 0};
  hipError_t e = hipSuccess;
  if (!rc) e = hipMemcpyAsync(h, m->d_res, 3 * sizeof(double), hipMemcpyDeviceToHost, s);
  const hipError_t e2 = hipFreeAsync(w, s);
  const hipError_t e3 = hipStreamSynchronize(s);
  if (rc) return rc;
  HIP_TRY(e);
  HIP_TRY(e2);
  HIP_TRY(e3);
  out[0] = 0.5 * h[0] + 0.5 * h[1];
  out[1] = 0.5 * h[0] + 0.5 * h[2];
  if (!std::isfinite(out[0]) || !std::isfinite(out[1])) return fail(DGM_ERR_UNSTABLE, "non-finite energy");
  return DGM_OK;
}

template <typename R>
int energy_var_impl(dgm_mesh* m, const R* E, const R* H, const R* Hn, double dt, double out[2], hipStream_t s) {
  const size_t nH = field_len(m, 1);
  int rc;
  if (!m->d_res) HIP_TRY(hipMalloc(&m->d_res, 4 * sizeof(double)));
  const R* Hq = Hn;
  R* hn = nullptr;
  if (!Hq) {
    HIP_TRY(hipMallocAsync(reinterpret_cast<void**>(&hn), nH * sizeof(R), s));
    rc = rate_impl<R>(m, E, hn, 0, s);
    if (!rc) {
      hipLaunchKernelGGL(xpay_kernel<R>, dim3(flat_blocks(nH)), dim3(kFlatThreads), 0, s, hn, H, nH, dt);
      if (hipGetLastError() != hipSuccess) rc = fail(DGM_ERR_HIP, "xpay kernel launch failed");
    }
    if (rc) {
      hipFreeAsync(hn, s);
      hipStreamSynchronize(s);
      return rc;
    }
    Hq = hn;
  }
  if (mass_built<double>(m->pE) && mass_built<double>(m->p))
    rc = energy_var_core<double, R>(m, E, H, Hq, out, s);
  else
    rc = energy_var_core<R, R>(m, E, H, Hq, out, s);
  if (hn) {
    const hipError_t e2 = hipFreeAsync(hn, s);
    const hipError_t e3 = hipStreamSynchronize(s);
    if (rc) return rc;
    HIP_TRY(e2);
    HIP_TRY(e3);
  }
  return rc;
}

int dense_ready(dgm_mesh* m, int prec, DenseOps** out) {
  const int q = prec == DGM_BF16 ? 0 : 1;
  if (!m->dense[q]) {
    const char* err = "";
    const int rc = dense_build(m->p, q, &m->dense[q], &err);
    if (rc) return fail(rc == -1 ? DGM_ERR_ARG : (rc == -5 ? DGM_ERR_OOM : DGM_ERR_HIP), err);
  }
  const size_t need = dense_scratch_floats(m->dense[q], m->K);
  if (m->jump_floats < need) {
    if (m->d_jump) HIP_TRY(hipFree(m->d_jump));
    m->d_jump = nullptr;
    m->jump_floats = 0;
    HIP_TRY(hipMalloc(&m->d_jump, need * sizeof(float)));
    m->jump_floats = need;
  }
  *out = m->dense[q];
  return DGM_OK;
}

int run_dense_phase(dgm_mesh* m, DenseOps* d, const float* U, float* V, int fld_u, double sdt, hipStream_t s) {
  HIP_TRY(dense_phase(d, U, V, m->d_M32[fld_u], m->d_nbr, (float)sdt, fld_u == 0 ? -1.f : 1.f, (int)m->K, m->d_jump, s));
  return DGM_OK;
}

int dense_rate(dgm_mesh* m, DenseOps* d, const float* in, float* out, int fld_u, hipStream_t s) {
  const size_t n = (size_t)3 * num_modes(m->p) * m->K;
  int rc;
  if ((rc = ensure_scratch(m, n * sizeof(float)))) return rc;
  float* tmp = static_cast<float*>(m->d_scratch);
  HIP_TRY(hipMemcpyAsync(tmp, in, n * sizeof(float), hipMemcpyDeviceToDevice, s));
  if ((rc = convert<float>(m, tmp, fld_u, true, s))) return rc;
  if ((rc = fill<float>(out, n, 0.f, s))) return rc;
  if ((rc = run_dense_phase(m, d, tmp, out, fld_u, fld_u == 0 ? -1.0 : 1.0, s))) return rc;
  return convert<float>(m, out, 1 - fld_u, false, s);
}


template <typename R>
int estimate_impl(dgm_mesh* m, double cfl, int iters, uint64_t seed, double* dt, double* rho_out, hipStream_t s) {
  int rc = DGM_OK;
  const size_t n = field_len(m, 1), nE = field_len(m, 0);  // x, z hold H; y holds E
  R* x = nullptr;
  HIP_TRY(hipMallocAsync(reinterpret_cast<void**>(&x), (2 * n + nE) * sizeof(R) + 5 * sizeof(double), s));
  R* const base = x;
  R* z = x + n;
  R* y = z + n;
  // three FP64 dot products after the vectors, aligned to 8 bytes
  double* d = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(y + nE) + 7) & ~uintptr_t(7));
  const unsigned blocks = flat_blocks(n);
  hipLaunchKernelGGL(splitmix_fill_kernel<R>, dim3(blocks), dim3(kFlatThreads), 0, s, x, n, (unsigned long long)seed);
  if (hipGetLastError() != hipSuccess) rc = fail(DGM_ERR_HIP, "start vector kernel launch failed");
  for (int it = 0; it < iters && !rc; ++it) {
    // z = dH(dE(x)) = -B x, where B = M_mu^{-1} C M_eps^{-1} C^T is similar to the
    // symmetric matrix of the bound; Rayleigh quotient in the M_mu inner product
    if ((rc = rate_impl<R>(m, x, y, 1, s))) break;
    if ((rc = rate_impl<R>(m, y, z, 0, s))) break;
    if ((rc = mdot<R>(m, x, z, 1, d + 0, s))) break;
    if ((rc = mdot<R>(m, x, x, 1, d + 1, s))) break;
    if ((rc = mdot<R>(m, z, z, 1, d + 2, s))) break;
    hipLaunchKernelGGL(scale_kernel<R>, dim3(blocks), dim3(kFlatThreads), 0, s, z, n, d + 2);
    if (hipGetLastError() != hipSuccess) rc = fail(DGM_ERR_HIP, "scale kernel launch failed");
    std::swap(x, z);
  }
  double h[3] = {0, 0, 0};
  hipError_t e = hipSuccess;
  if (!rc) e = hipMemcpyAsync(h, d, 3 * sizeof(double), hipMemcpyDeviceToHost, s);
  const hipError_t e2 = hipFreeAsync(base, s);  // freed on every path
  const hipError_t e3 = hipStreamSynchronize(s);
  if (rc) return rc;
  HIP_TRY(e);
  HIP_TRY(e2);
  HIP_TRY(e3);
  const double rho = -h[0] / h[1];
  if (!(rho > 0.0) || !std::isfinite(rho)) return fail(DGM_ERR_UNSTABLE, "power iteration did not give a positive estimate");
  if (rho_out) *rho_out = rho;
  *dt = cfl * 2.0 / std::sqrt(rho);
  return DGM_OK;
}

// The same power iteration with the approximate mass inverses (material linear on the
// elements).  B = P_mu C P_eps C^T is self-adjoint in the inner product of
// M~_mu = P_mu^{-1}, and with x = P_mu y that product is (x, x') = (y, G x') (G the
// unit-material metric), so the iteration carries y beside x instead of solving:
// w = unit-material dH(dE(x)) gives z = B x = P_mu w with z = P_mu w, i.e. the y of z is w.
template <typename R>
int estimate_var_impl(dgm_mesh* m, double cfl, int iters, uint64_t seed, double* dt, double* rho_out, hipStream_t s) {
  int rc = DGM_OK;
  const size_t n = field_len(m, 1), nE = field_len(m, 0);  // x, z, y, w hold H; v holds E
  R* x = nullptr;
  HIP_TRY(hipMallocAsync(reinterpret_cast<void**>(&x), (4 * n + nE) * sizeof(R) + 5 * sizeof(double), s));
  R* const base = x;
  R* z = x + n;
  R* y = z + n;
  R* w = y + n;
  R* v = w + n;
  double* d = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(v + nE) + 7) & ~uintptr_t(7));
  const unsigned blocks = flat_blocks(n);
  hipLaunchKernelGGL(splitmix_fill_kernel<R>, dim3(blocks), dim3(kFlatThreads), 0, s, y, n, (unsigned long long)seed);
  if (hipGetLastError() != hipSuccess) rc = fail(DGM_ERR_HIP, "start vector kernel launch failed");
  if (!rc) rc = run_mass<R>(m, y, x, 1, 1.0, false, s);
  for (int it = 0; it < iters && !rc; ++it) {
    if ((rc = rate_impl<R>(m, x, v, 1, s))) break;
    if ((rc = rate_impl<R>(m, v, w, 0, s, nullptr, 0.0, false))) break;
    if ((rc = run_mass<R>(m, w, z, 1, 1.0, false, s))) break;
    if ((rc = mdot<R>(m, y, z, 1, d + 0, s))) break;
    if ((rc = mdot<R>(m, y, x, 1, d + 1, s))) break;
    if ((rc = mdot<R>(m, w, z, 1, d + 2, s))) break;
    hipLaunchKernelGGL(scale_kernel<R>, dim3(blocks), dim3(kFlatThreads), 0, s, z, n, d + 2);
    hipLaunchKernelGGL(scale_kernel<R>, dim3(blocks), dim3(kFlatThreads), 0, s, w, n, d + 2);
    if (hipGetLastError() != hipSuccess) rc = fail(DGM_ERR_HIP, "scale kernel launch failed");
    std::swap(x, z);
    std::swap(y, w);
  }
  double h[3] = {0, 0, 0};
  hipError_t e = hipSuccess;
  if (!rc) e = hipMemcpyAsync(h, d, 3 * sizeof(double), hipMemcpyDeviceToHost, s);
  const hipError_t e2 = hipFreeAsync(base, s);
  const hipError_t e3 = hipStreamSynchronize(s);
  if (rc) return rc;
  HIP_TRY(e);
  HIP_TRY(e2);
  HIP_TRY(e3);
  const double rho = -h[0] / h[1];
  if (!(rho > 0.0) || !std::isfinite(rho)) return fail(DGM_ERR_UNSTABLE, "power iteration did not give a positive estimate");
  if (rho_out) *rho_out = rho;
  *dt = cfl * 2.0 / std::sqrt(rho);
  return DGM_OK;
}

// Face data of the stabilised flux for the current order: per element side that owns its
// face (a wall side, or the side of the smaller element index) with sorted-vertex edge
// vectors t_1, t_2 of the face, outward unit normal nu, area |F| and Gram matrix G:
// the update matrix C = -(alpha/h_F) c, nu x t_k = sum_i c[k][i] t_i (16,K: 4 per face),
// and the energy weight (h_F/alpha) 2|F| G^{-1} (12,K: 3 per face), with
// h_F = 3 min |T| / |F| over the face's elements and alpha = alpha0 p^2 (FP64 on the host).
int stab_ready(dgm_mesh* m) {
  if (!(m->stab_alpha0 > 0.0)) return fail(DGM_ERR_STATE, "stabilised flux not set (dgm_set_stab_alpha)");
  if (m->d_stab && m->stab_p == m->p) return DGM_OK;
  const int64_t K = m->K;
  const size_t Ks = (size_t)K;
  const double alpha = m->stab_alpha0 * m->p * m->p;
  std::vector<float> sc32(16 * Ks, 0.f);
  std::vector<double> sc64(16 * Ks, 0.0), wf(12 * Ks, 0.0);
  for (int64_t e = 0; e < K; ++e) {
    double P[4][3] = {{0, 0, 0}};
    for (int q = 1; q < 4; ++q)
      for (int d = 0; d < 3; ++d) P[q][d] = m->F[9 * e + 3 * d + (q - 1)];
    for (int f = 0; f < 4; ++f) {
      const int code = m->nbr[f * Ks + e];
      const int64_t nb = code >= 0 ? code >> 2 : -1;
      if (code >= 0 && nb < e) continue;  // the neighbour owns this face
      int w[3], c = 0;
      for (int q = 0; q < 4; ++q)
        if (q != f) w[c++] = q;
      double t[2][3], n[3];
      for (int d = 0; d < 3; ++d) {
        t[0][d] = P[w[1]][d] - P[w[0]][d];
        t[1][d] = P[w[2]][d] - P[w[0]][d];
      }
      n[0] = t[0][1] * t[1][2] - t[0][2] * t[1][1];
      n[1] = t[0][2] * t[1][0] - t[0][0] * t[1][2];
      n[2] = t[0][0] * t[1][1] - t[0][1] * t[1][0];
      const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      double out = 0.0;
      for (int d = 0; d < 3; ++d) out += n[d] * (P[f][d] - P[w[0]][d]);
      const double sgn = out > 0.0 ? -1.0 : 1.0;  // away from the opposite vertex
      double nu[3];
      for (int d = 0; d < 3; ++d) nu[d] = sgn * n[d] / nn;
      const double area = 0.5 * nn;
      double G[2][2];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) G[a][b] = t[a][0] * t[b][0] + t[a][1] * t[b][1] + t[a][2] * t[b][2];
      const double det = G[0][0] * G[1][1] - G[0][1] * G[1][0];
      const double Gi[2][2] = {{G[1][1] / det, -G[0][1] / det}, {-G[1][0] / det, G[0][0] / det}};
      const double Je = std::fabs(m->J[e]);
      const double hF = (code >= 0 ? std::min(Je, std::fabs(m->J[nb])) : Je) / (2.0 * area);
      for (int k = 0; k < 2; ++k) {
        double v[3] = {nu[1] * t[k][2] - nu[2] * t[k][1], nu[2] * t[k][0] - nu[0] * t[k][2],
                       nu[0] * t[k][1] - nu[1] * t[k][0]};
        double r[2];
        for (int i = 0; i < 2; ++i) r[i] = t[i][0] * v[0] + t[i][1] * v[1] + t[i][2] * v[2];
        for (int i = 0; i < 2; ++i) {
          const double cki = Gi[i][0] * r[0] + Gi[i][1] * r[1];
          const double Cv = -(alpha / hF) * cki;
          sc64[(4 * f + 2 * k + i) * Ks + e] = Cv;
          sc32[(4 * f + 2 * k + i) * Ks + e] = (float)Cv;
        }
      }
      const double sw = (hF / alpha) * 2.0 * area;
      wf[(3 * f + 0) * Ks + e] = sw * Gi[0][0];
      wf[(3 * f + 1) * Ks + e] = sw * Gi[0][1];
      wf[(3 * f + 2) * Ks + e] = sw * Gi[1][1];
    }
  }
  const size_t b32 = (16 * Ks * sizeof(float) + 255) & ~size_t(255);
  const size_t b64 = (16 * Ks * sizeof(double) + 255) & ~size_t(255);
  if (!m->d_stab) HIP_TRY(hipMalloc(&m->d_stab, b32 + b64 + 12 * Ks * sizeof(double)));
  char* base = static_cast<char*>(m->d_stab);
  m->d_SC32 = reinterpret_cast<float*>(base);
  m->d_SC64 = reinterpret_cast<double*>(base + b32);
  m->d_WF = reinterpret_cast<double*>(base + b32 + b64);
  HIP_TRY(hipMemcpy(m->d_SC32, sc32.data(), sc32.size() * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(m->d_SC64, sc64.data(), sc64.size() * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(m->d_WF, wf.data(), wf.size() * sizeof(double), hipMemcpyHostToDevice));
  m->stab_p = m->p;
  return DGM_OK;
}

size_t face_unknowns(const dgm_mesh* m) { return (size_t)8 * num_face_modes(m->p) * (size_t)m->K; }

template <typename R>
int fdot(dgm_mesh* m, const R* A, const R* B, double* d_out, hipStream_t s) {
  const int nb = (int)((m->K + kRedThreads - 1) / kRedThreads);
  int rc;
  if ((rc = ensure_partial(m, nb))) return rc;
  hipLaunchKernelGGL(fdot_partial_kernel<R>, dim3(nb), dim3(kRedThreads), 0, s, A, B, m->d_WF,
                     num_face_modes(m->p), (int)m->K, m->d_partial);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(kRedThreads), 0, s, m->d_partial, nb, d_out);
  HIP_TRY(hipGetLastError());
  return DGM_OK;
}

// dH and dHF from E (either may be null), dE from H and HF.
template <typename R>
int apply_stab_impl(dgm_mesh* m, const R* E, const R* H, const R* HF, R* dE, R* dH, R* dHF, hipStream_t s) {
  const size_t n = (size_t)3 * num_modes(m->p) * m->K;
  int rc;
  if (dH || dHF) {
    R* outH = dH;
    if (!outH) {
      if ((rc = ensure_scratch(m, 2 * n * sizeof(R)))) return rc;
      outH = static_cast<R*>(m->d_scratch) + n;  // the rate's copy of E uses the first half
    }
    if (dHF && (rc = fill<R>(dHF, face_unknowns(m), (R)0, s))) return rc;
    if ((rc = rate_impl<R>(m, E, outH, 0, s, dHF, 1.0))) return rc;
  }
  if (dE && (rc = rate_impl<R>(m, H, dE, 1, s, const_cast<R*>(HF), 0.0))) return rc;
  return DGM_OK;
}

// W and Q with the face term: central parts from energy_impl, then
// 1/2 (HF, W HF) and 1/2 (HF, W HF_next) with HF_next = HF + dt dHF(E).
template <typename R>
int energy_stab_impl(dgm_mesh* m, const R* E, const R* H, const R* HF, double dt, double out[2], hipStream_t s) {
  int rc;
  if ((rc = energy_impl<R>(m, E, H, dt == 0.0 ? H : nullptr, dt, out, s))) return rc;
  const size_t n = (size_t)3 * num_modes(m->p) * m->K, nh = face_unknowns(m);
  R* hn = nullptr;
  HIP_TRY(hipMallocAsync(reinterpret_cast<void**>(&hn), nh * sizeof(R), s));
  rc = DGM_OK;
  if (dt != 0.0) {
    if ((rc = ensure_scratch(m, 2 * n * sizeof(R))) == DGM_OK) {
      if (hipMemcpyAsync(hn, HF, nh * sizeof(R), hipMemcpyDeviceToDevice, s) != hipSuccess)
        rc = fail(DGM_ERR_HIP, "face unknown copy failed");
      if (!rc) rc = rate_impl<R>(m, E, static_cast<R*>(m->d_scratch) + n, 0, s, hn, dt);
    }
  }
  if (!rc) rc = fdot<R>(m, HF, HF, m->d_res + 0, s);
  if (!rc) rc = fdot<R>(m, HF, dt != 0.0 ? hn : HF, m->d_res + 1, s);
  double h[2] = {0, 0};
  hipError_t e = hipSuccess;
  if (!rc) e = hipMemcpyAsync(h, m->d_res, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
  const hipError_t e2 = hipFreeAsync(hn, s);
  const hipError_t e3 = hipStreamSynchronize(s);
  if (rc) return rc;
  HIP_TRY(e);
  HIP_TRY(e2);
  HIP_TRY(e3);
  out[0] += 0.5 * h[0];
  out[1] += 0.5 * h[1];
  if (!std::isfinite(out[0]) || !std::isfinite(out[1])) return fail(DGM_ERR_UNSTABLE, "non-finite energy");
  return DGM_OK;
}

// Power iteration on E -> -dE(dH(E), dHF(E)) (the stabilised second-order operator),
// Rayleigh quotient in the M_eps inner product.
template <typename R>
int estimate_stab_impl(dgm_mesh* m, double cfl, int iters, uint64_t seed, double* dt, double* rho_out, hipStream_t s) {
  int rc = DGM_OK;
  const size_t n = (size_t)3 * num_modes(m->p) * m->K, nh = face_unknowns(m);
  R* x = nullptr;
  HIP_TRY(hipMallocAsync(reinterpret_cast<void**>(&x), (3 * n + nh) * sizeof(R) + 5 * sizeof(double), s));
  R* const base = x;
  R* y = x + n;
  R* z = y + n;
  R* yf = z + n;
  double* d = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(yf + nh) + 7) & ~uintptr_t(7));
  const unsigned blocks = flat_blocks(n);
  hipLaunchKernelGGL(splitmix_fill_kernel<R>, dim3(blocks), dim3(kFlatThreads), 0, s, x, n, (unsigned long long)seed);
  if (hipGetLastError() != hipSuccess) rc = fail(DGM_ERR_HIP, "start vector kernel launch failed");
  for (int it = 0; it < iters && !rc; ++it) {
    if ((rc = apply_stab_impl<R>(m, x, nullptr, nullptr, nullptr, y, yf, s))) break;
    if ((rc = apply_stab_impl<R>(m, nullptr, y, yf, z, nullptr, nullptr, s))) break;
    if ((rc = mdot<R>(m, x, z, 0, d + 0, s))) break;
    if ((rc = mdot<R>(m, x, x, 0, d + 1, s))) break;
    if ((rc = mdot<R>(m, z, z, 0, d + 2, s))) break;
    hipLaunchKernelGGL(scale_kernel<R>, dim3(blocks), dim3(kFlatThreads), 0, s, z, n, d + 2);
    if (hipGetLastError() != hipSuccess) rc = fail(DGM_ERR_HIP, "scale kernel launch failed");
    std::swap(x, z);
  }
  double h[3] = {0, 0, 0};
  hipError_t e = hipSuccess;
  if (!rc) e = hipMemcpyAsync(h, d, 3 * sizeof(double), hipMemcpyDeviceToHost, s);
  const hipError_t e2 = hipFreeAsync(base, s);
  const hipError_t e3 = hipStreamSynchronize(s);
  if (rc) return rc;
  HIP_TRY(e);
  HIP_TRY(e2);
  HIP_TRY(e3);
  const double rho = -h[0] / h[1];
  if (!(rho > 0.0) || !std::isfinite(rho)) return fail(DGM_ERR_UNSTABLE, "power iteration did not give a positive estimate");
  if (rho_out) *rho_out = rho;
  *dt = cfl * 2.0 / std::sqrt(rho);
  return DGM_OK;
}

}  // namespace

// ---------------------------------------------------------------- C-ABI
extern "C" {

const char* dgm_last_error(void) { return g_err.c_str(); }

int dgm_num_modes(int p) { return p < 0 ? 0 : num_modes(p); }
int dgm_num_face_modes(int p) { return p < 0 ? 0 : (p + 1) * (p + 2) / 2; }
int dgm_max_order(int dtype) { return dtype == DGM_F64 ? DGM_MAX_ORDER_F64 : DGM_MAX_ORDER_F32; }

int dgm_mode_index(int p, int m, int* i, int* j, int* k) {
  if (p < 0 || m < 0 || m >= num_modes(p) || !i || !j || !k) return fail(DGM_ERR_ARG, "mode index out of range");
  int r = 0;
  for (int n = 0; n <= p; ++n)
    for (int a = 0; a <= n; ++a)
      for (int b = 0; b <= n - a; ++b, ++r)
        if (r == m) {
          *i = a;
          *j = b;
          *k = n - a - b;
          return DGM_OK;
        }
  return fail(DGM_ERR_ARG, "mode index out of range");
}

int dgm_create_mesh(const double* verts, int64_t nv, const int64_t* tets, int64_t nt, dgm_mesh** out) {
  if (!verts || !tets || !out || nv < 4 || nt < 1) return fail(DGM_ERR_ARG, "bad mesh arguments");
  // neighbour codes 4 e + f stay in int32, and a per-tile launch of up to 1024
  // threads per 64 elements stays below 2^32 work-items
  if (nt > kMaxElements) return fail(DGM_ERR_ARG, "too many elements (max " + std::to_string(kMaxElements) + ")");
  *out = nullptr;
  auto* m = new dgm_mesh();
  m->K = nt;
  m->F.resize(9 * nt);
  m->J.resize(nt);
  std::vector<int64_t> sorted(4 * nt);
  m->perm.resize(4 * nt);
  for (int64_t e = 0; e < nt; ++e) {
    int64_t v[4];
    for (int q = 0; q < 4; ++q) {
      v[q] = tets[4 * e + q];
      if (v[q] < 0 || v[q] >= nv) {
        delete m;
        return fail(DGM_ERR_ARG, "vertex id out of range in element " + std::to_string(e));
      }
    }
    std::sort(v, v + 4);
    if (v[0] == v[1] || v[1] == v[2] || v[2] == v[3]) {
      delete m;
      return fail(DGM_ERR_MESH_DEGENERATE, "repeated vertex in element " + std::to_string(e));
    }
    for (int q = 0; q < 4; ++q)
      for (int c = 0; c < 4; ++c)
        if (tets[4 * e + c] == v[q]) m->perm[4 * e + q] = (unsigned char)c;
    double P[4][3], h = 0.0;
    for (int q = 0; q < 4; ++q) {
      sorted[4 * e + q] = v[q];
      for (int d = 0; d < 3; ++d) P[q][d] = verts[3 * v[q] + d];
    }
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b) {
        double l2 = 0.0;
        for (int d = 0; d < 3; ++d) l2 += (P[a][d] - P[b][d]) * (P[a][d] - P[b][d]);
        h = std::max(h, std::sqrt(l2));
      }
    double Fm[3][3];
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 3; ++c) Fm[d][c] = P[c + 1][d] - P[0][d];
    const double J = Fm[0][0] * (Fm[1][1] * Fm[2][2] - Fm[1][2] * Fm[2][1]) -
                     Fm[0][1] * (Fm[1][0] * Fm[2][2] - Fm[1][2] * Fm[2][0]) +
                     Fm[0][2] * (Fm[1][0] * Fm[2][1] - Fm[1][1] * Fm[2][0]);
    if (!(std::fabs(J) >= 1e-12 * h * h * h) || !std::isfinite(J)) {
      delete m;
      return fail(DGM_ERR_MESH_DEGENERATE, "degenerate element " + std::to_string(e));
    }
    std::memcpy(&m->F[9 * e], Fm, sizeof(Fm));
    m->J[e] = J;
  }
  // faces: local face f is opposite local vertex f; key = its sorted vertex triple
  struct FaceRec {
    int64_t a, b, c;
    int64_t e;
    int f;
  };
  std::vector<FaceRec> recs;
  recs.reserve(4 * nt);
  for (int64_t e = 0; e < nt; ++e)
    for (int f = 0; f < 4; ++f) {
      int64_t id[3];
      int q = 0;
      for (int v = 0; v < 4; ++v)
        if (v != f) id[q++] = sorted[4 * e + v];
      recs.push_back({id[0], id[1], id[2], e, f});
    }
  // order by (a, b, c, e): a counting sort on the smallest id a (O(nt + nv)), then each
  // group sharing a vertex (a few dozen faces) by the other two ids
  std::vector<int64_t> start(nv + 1, 0);
  for (const FaceRec& r : recs) ++start[r.a + 1];
  for (int64_t v = 0; v < nv; ++v) start[v + 1] += start[v];
  std::vector<FaceRec> faces(recs.size());
  {
    std::vector<int64_t> pos(start.begin(), start.end() - 1);
    for (const FaceRec& r : recs) faces[pos[r.a]++] = r;
  }
  recs = std::vector<FaceRec>();
  for (int64_t v = 0; v < nv; ++v)
    if (start[v + 1] - start[v] > 1)
      std::sort(faces.begin() + start[v], faces.begin() + start[v + 1], [](const FaceRec& x, const FaceRec& y) {
        if (x.b != y.b) return x.b < y.b;
        if (x.c != y.c) return x.c < y.c;
        return x.e < y.e;
      });
  m->nbr.assign(4 * nt, -1);
  for (size_t s = 0; s < faces.size();) {
    size_t t = s + 1;
    while (t < faces.size() && faces[t].a == faces[s].a && faces[t].b == faces[s].b && faces[t].c == faces[s].c) ++t;
    if (t - s > 2) {
      delete m;
      return fail(DGM_ERR_MESH_NONMANIFOLD, "face shared by more than two elements");
    }
    if (t - s == 2) {
      const FaceRec &x = faces[s], &y = faces[s + 1];
      if (x.e == y.e) {
        delete m;
        return fail(DGM_ERR_MESH_DEGENERATE, "element touches itself");
      }
      m->nbr[x.f * nt + x.e] = (int)(y.e * 4 + y.f);
      m->nbr[y.f * nt + y.e] = (int)(x.e * 4 + x.f);
    }
    s = t;
  }
  geom_layout(nt, m->geom_off);
  const hipError_t ea = hipMalloc(&m->d_geom, m->geom_off[kGeomArrays]);
  if (ea != hipSuccess) {
    m->d_geom = nullptr;
    dgm_destroy(m);
    return fail(ea == hipErrorOutOfMemory ? DGM_ERR_OOM : DGM_ERR_HIP,
                std::string("hipMalloc (mesh block): ") + hipGetErrorString(ea));
  }
  {
    unsigned char* base = static_cast<unsigned char*>(m->d_geom);
    const size_t* off = m->geom_off;
    m->d_nbr = reinterpret_cast<int*>(base + off[kNbr]);
    for (int f = 0; f < 2; ++f) {
      m->d_M32[f] = reinterpret_cast<float*>(base + off[kM32E + f]);
      m->d_Minv32[f] = reinterpret_cast<float*>(base + off[kMinv32E + f]);
      m->d_M64[f] = reinterpret_cast<double*>(base + off[kM64E + f]);
      m->d_Minv64[f] = reinterpret_cast<double*>(base + off[kMinv64E + f]);
      m->d_G[f] = reinterpret_cast<double*>(base + off[kGE + f]);
    }
  }
  const hipError_t ec = hipMemcpy(m->d_nbr, m->nbr.data(), m->nbr.size() * sizeof(int), hipMemcpyHostToDevice);
  int rc = ec == hipSuccess ? DGM_OK : fail(DGM_ERR_HIP, std::string("hipMemcpy (neighbours): ") + hipGetErrorString(ec));
  if (!rc) rc = material_impl(m, nullptr, nullptr);
  if (rc) {
    dgm_destroy(m);
    return rc;
  }
  *out = m;
  return DGM_OK;
}

int dgm_destroy(dgm_mesh* m) {
  if (!m) return DGM_OK;
  hipFree(m->d_geom);  // the neighbour codes and every per-element factor
  hipFree(m->d_scratch);
  hipFree(m->d_T);
  hipFree(m->d_partial);
  hipFree(m->d_res);
  dense_free(m->dense[0]);
  dense_free(m->dense[1]);
  hipFree(m->d_jump);
  hipFree(m->d_stab);
  hipFree(m->d_var);
  delete m;
  return DGM_OK;
}

int dgm_num_elements(const dgm_mesh* m, int64_t* K) {
  if (!m || !K) return fail(DGM_ERR_ARG, "null argument");
  *K = m->K;
  return DGM_OK;
}

int dgm_set_order(dgm_mesh* m, int p) {
  if (!m) return fail(DGM_ERR_ARG, "null mesh");
  if (!order_built(p, DGM_F32)) return fail(DGM_ERR_ARG, "order " + std::to_string(p) + " not built");
  if (m->p != p) {
    for (int q = 0; q < 2; ++q) {
      dense_free(m->dense[q]);
      m->dense[q] = nullptr;
    }
  }
  m->p = p;
  m->pE = p;
  return DGM_OK;
}

int dgm_set_orders(dgm_mesh* m, int pE, int pH) {
  if (!m) return fail(DGM_ERR_ARG, "null mesh");
  if (pE != pH && pE != pH + 1) return fail(DGM_ERR_ARG, "E's order must equal H's or exceed it by one");
  if (pE == pH) return dgm_set_order(m, pH);
  if (!mixed_built(pH, DGM_F32))
    return fail(DGM_ERR_ARG, "mixed orders (" + std::to_string(pE) + ", " + std::to_string(pH) + ") not built");
  int rc;
  if ((rc = dgm_set_order(m, pH))) return rc;
  m->pE = pE;
  return DGM_OK;
}

int dgm_orders(const dgm_mesh* m, int* pE, int* pH) {
  if (!m || !pE || !pH) return fail(DGM_ERR_ARG, "null argument");
  *pE = m->pE;
  *pH = m->p;
  return DGM_OK;
}

int dgm_set_check_interval(dgm_mesh* m, int64_t every) {
  if (!m || every < 0) return fail(DGM_ERR_ARG, "bad check interval");
  m->check_every = every;
  return DGM_OK;
}

int dgm_set_material(dgm_mesh* m, const double* eps, const double* mu) {
  if (!m) return fail(DGM_ERR_ARG, "null mesh");
  const int rc = material_impl(m, eps, mu);
  if (!rc) m->varmat = false;
  return rc;
}

int dgm_apply_mass_inverse(dgm_mesh* m, int dtype, int field, const void* X, void* Y, hipStream_t s) {
  int rc = check_order(m, dtype);
  if (rc) return rc;
  if (!m->varmat) return fail(DGM_ERR_STATE, "no material linear on the elements (dgm_set_material_linear)");
  if (field != 0 && field != 1) return fail(DGM_ERR_ARG, "field must be 0 (E, eps) or 1 (H, mu)");
  if (!X || !Y || X == Y) return fail(DGM_ERR_ARG, "X and Y must be distinct device arrays");
  if (dtype == DGM_F32) return run_mass<float>(m, (const float*)X, (float*)Y, field, 1.0, false, s);
  return run_mass<double>(m, (const double*)X, (double*)Y, field, 1.0, false, s);
}

int dgm_set_material_linear(dgm_mesh* m, const double* eps, const double* mu) {
  if (!m) return fail(DGM_ERR_ARG, "null mesh");
  const size_t K = (size_t)m->K;
  // host images: eps then mu, (4,K) each at the sorted vertices, FP32 block then FP64
  std::vector<float> v32(8 * K);
  std::vector<double> v64(8 * K);
  for (int fld = 0; fld < 2; ++fld) {
    const double* src = fld == 0 ? eps : mu;
    for (size_t e = 0; e < K; ++e)
      for (int q = 0; q < 4; ++q) {
        const double c = src ? src[4 * e + m->perm[4 * e + q]] : 1.0;
        if (!(c > 0.0) || !std::isfinite(c))
          return fail(DGM_ERR_MATERIAL, "material value must be finite and > 0 (element " + std::to_string(e) + ")");
        v64[(4 * fld + q) * K + e] = c;
        v32[(4 * fld + q) * K + e] = (float)c;
      }
  }
  const size_t b32 = (8 * K * sizeof(float) + 255) & ~size_t(255);
  if (!m->d_var) HIP_TRY(hipMalloc(&m->d_var, b32 + 8 * K * sizeof(double)));
  char* base = static_cast<char*>(m->d_var);
  HIP_TRY(hipMemcpy(base, v32.data(), v32.size() * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(base + b32, v64.data(), v64.size() * sizeof(double), hipMemcpyHostToDevice));
  for (int fld = 0; fld < 2; ++fld) {
    m->d_var32[fld] = reinterpret_cast<float*>(base) + 4 * fld * K;
    m->d_var64[fld] = reinterpret_cast<double*>(base + b32) + 4 * fld * K;
  }
  const int rc = material_impl(m, nullptr, nullptr);  // unit-material metrics
  m->varmat = rc == DGM_OK;
  return rc;
}

int dgm_apply_curl(dgm_mesh* m, int dtype, const void* E, const void* H, void* dE, void* dH, hipStream_t s) {
  int rc = check_order(m, dtype);
  if (rc) return rc;
  if ((dH && !E) || (dE && !H)) return fail(DGM_ERR_ARG, "output requested without its input");
  if ((dH && (dH == E || dH == H)) || (dE && (dE == E || dE == H))) return fail(DGM_ERR_ARG, "outputs alias inputs");
  if (dtype == DGM_F32) {
    if (dH && (rc = rate_impl<float>(m, (const float*)E, (float*)dH, 0, s))) return rc;
    if (dE && (rc = rate_impl<float>(m, (const float*)H, (float*)dE, 1, s))) return rc;
  } else {
    if (dH && (rc = rate_impl<double>(m, (const double*)E, (double*)dH, 0, s))) return rc;
    if (dE && (rc = rate_impl<double>(m, (const double*)H, (double*)dE, 1, s))) return rc;
  }
  return DGM_OK;
}

int dgm_step(dgm_mesh* m, int dtype, void* E, void* H, double dt, int64_t nsteps, hipStream_t s) {
  int rc = check_order(m, dtype);
  if (rc) return rc;
  if (!E || !H || E == H || nsteps < 0 || !std::isfinite(dt)) return fail(DGM_ERR_ARG, "bad step arguments");
  if (nsteps == 0) return DGM_OK;
  const bool red = m->check_every > 0;
  if (dtype == DGM_F32) {
    StepWork<float> ws;
    if ((rc = mesh_work<float>(m, red, &ws))) return rc;
    return step_impl<float>(m, (float*)E, (float*)H, dt, nsteps, s, ws);
  }
  StepWork<double> ws;
  if ((rc = mesh_work<double>(m, red, &ws))) return rc;
  return step_impl<double>(m, (double*)E, (double*)H, dt, nsteps, s, ws);
}

int dgm_step_probe(dgm_mesh* m, int dtype, void* E, void* H, double dt, int64_t nsteps, const void* w,
                   double* signal, hipStream_t s) {
  int rc = check_order(m, dtype);
  if (rc) return rc;
  if (!E || !H || E == H || !w || !signal || nsteps < 0 || !std::isfinite(dt))
    return fail(DGM_ERR_ARG, "bad step_probe arguments");
  if (nsteps == 0) return DGM_OK;
  double* d_sig = nullptr;
  HIP_TRY(hipMallocAsync(reinterpret_cast<void**>(&d_sig), (size_t)nsteps * sizeof(double), s));
  if (dtype == DGM_F32) {
    StepWork<float> ws;
    rc = mesh_work<float>(m, true, &ws);
    if (!rc) rc = step_impl<float>(m, (float*)E, (float*)H, dt, nsteps, s, ws, (const float*)w, d_sig);
  } else {
    StepWork<double> ws;
    rc = mesh_work<double>(m, true, &ws);
    if (!rc) rc = step_impl<double>(m, (double*)E, (double*)H, dt, nsteps, s, ws, (const double*)w, d_sig);
  }
  hipError_t e = hipSuccess;
  if (!rc) e = hipMemcpyAsync(signal, d_sig, (size_t)nsteps * sizeof(double), hipMemcpyDeviceToHost, s);
  const hipError_t e2 = hipFreeAsync(d_sig, s);  // freed on every path
  const hipError_t e3 = hipStreamSynchronize(s);
  if (rc) return rc;
  HIP_TRY(e);
  HIP_TRY(e2);
  HIP_TRY(e3);
  return DGM_OK;
}

int dgm_set_stab_alpha(dgm_mesh* m, double alpha0) {
  if (!m) return fail(DGM_ERR_ARG, "null mesh");
  if (!(alpha0 > 0.0) || !std::isfinite(alpha0)) return fail(DGM_ERR_ARG, "alpha0 must be positive and finite");
  m->stab_alpha0 = alpha0;
  m->stab_p = 0;  // face data rebuilt on the next stabilised call
  return DGM_OK;
}

int dgm_num_face_unknowns(const dgm_mesh* m, int64_t* n) {
  if (!m || !n) return fail(DGM_ERR_ARG, "null argument");
  if (m->p < 1) return fail(DGM_ERR_STATE, "order not set (dgm_set_order)");
  *n = (int64_t)face_unknowns(m);
  return DGM_OK;
}

int dgm_apply_stab(dgm_mesh* m, int dtype, const void* E, const void* H, const void* HF, void* dE, void* dH, void* dHF,
                   hipStream_t s) {
  int rc = check_order(m, dtype);
  if (rc) return rc;
  if ((rc = check_equal_orders(m, "the stabilised flux"))) return rc;
  if ((rc = stab_ready(m))) return rc;
  if ((rc = check_constant_material(m, "the stabilised flux"))) return rc;
  if (((dH || dHF) && !E) || (dE && (!H || !HF))) return fail(DGM_ERR_ARG, "output requested without its input");
  const void* outs[3] = {dE, dH, dHF};
  for (const void* o : outs)
    if (o && (o == E || o == H || o == HF)) return fail(DGM_ERR_ARG, "outputs alias inputs");
  if (dtype == DGM_F32)
    return apply_stab_impl<float>(m, (const float*)E, (const float*)H, (const float*)HF, (float*)dE, (float*)dH,
                                  (float*)dHF, s);
  return apply_stab_impl<double>(m, (const double*)E, (const double*)H, (const double*)HF, (double*)dE, (double*)dH,
                                 (double*)dHF, s);
}

int dgm_step_stab(dgm_mesh* m, int dtype, void* E, void* H, void* HF, double dt, int64_t nsteps, hipStream_t s) {
  int rc = check_order(m, dtype);
  if (rc) return rc;
  if ((rc = check_equal_orders(m, "the stabilised flux"))) return rc;
  if ((rc = stab_ready(m))) return rc;
  if ((rc = check_constant_material(m, "the stabilised flux"))) return rc;
  if (!E || !H || !HF || E == H || E == HF || H == HF || nsteps < 0 || !std::isfinite(dt))
    return fail(DGM_ERR_ARG, "bad step arguments");
  if (nsteps == 0) return DGM_OK;
  const bool red = m->check_every > 0;
  if (dtype == DGM_F32) {
    StepWork<float> ws;
    if ((rc = mesh_work<float>(m, red, &ws))) return rc;
    return step_impl<float>(m, (float*)E, (float*)H, dt, nsteps, s, ws, nullptr, nullptr, (float*)HF);
  }
  StepWork<double> ws;
  if ((rc = mesh_work<double>(m, red, &ws))) return rc;
  return step_impl<double>(m, (double*)E, (double*)H, dt, nsteps, s, ws, nullptr, nullptr, (double*)HF);
}

int dgm_energy_stab(dgm_mesh* m, int dtype, const void* E, const void* H, const void* HF, double dt, double out[2],
                    hipStream_t s) {
  int rc = check_order(m, dtype);
  if (rc) return rc;
  if ((rc = check_equal_orders(m, "the stabilised flux"))) return rc;
  if ((rc = stab_ready(m))) return rc;
  if ((rc = check_constant_material(m, "the stabilised flux"))) return rc;
  if (!E || !H || !HF || !out || !std::isfinite(dt)) return fail(DGM_ERR_ARG, "bad energy arguments");
  return dtype == DGM_F32 ? energy_stab_impl<float>(m, (const float*)E, (const float*)H, (const float*)HF, dt, out, s)
                          : energy_stab_impl<double>(m, (const double*)E, (const double*)H, (const double*)HF, dt, out, s);
}

int dgm_estimate_dt_stab(dgm_mesh* m, double cfl, int iters, uint64_t seed, double* dt, double* rho_out,
                         hipStream_t s) {
  int rc = check_order(m, DGM_F32);
  if (rc) return rc;
  if ((rc = check_equal_orders(m, "the stabilised flux"))) return rc;
  if ((rc = stab_ready(m))) return rc;
  if ((rc = check_constant_material(m, "the stabilised flux"))) return rc;
  if (!dt || iters < 1 || !(cfl > 0.0)) return fail(DGM_ERR_ARG, "bad estimate_dt arguments");
  return m->p <= DGM_MAX_ORDER_F64 ? estimate_stab_impl<double>(m, cfl, iters, seed, dt, rho_out, s)
                                   : estimate_stab_impl<float>(m, cfl, iters, seed, dt, rho_out, s);
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free step
// Workspace of dgm_step_noalloc: a file-scope device array, one copy per GPU the library
// runs on, held until the process ends.  In host code `scratch` names a host-side stand-in,
// not the device memory: its device address is resolved once per device with
// hipGetSymbolAddress (with that device current) and only that address is passed on.
static __device__ __align__(256) unsigned char scratch[DGM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// Device address of `scratch` on the current device (resolved on the first call there).
int scratch_address(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices) return fail(DGM_ERR_ARG, "device index beyond the workspace table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(DGM_ERR_HIP, "hipGetSymbolAddress returned a null workspace address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return DGM_OK;
}

constexpr size_t kScratchPartialOff = 0;                                         // kDotBlocks doubles
constexpr size_t kScratchResOff = kScratchPartialOff + kDotBlocks * sizeof(double);  // 2 doubles
constexpr size_t kScratchTraceOff = (kScratchResOff + 2 * sizeof(double) + 255) & ~size_t(255);

// Bytes of the workspace a run on mesh m in precision rsize needs.
size_t noalloc_bytes(const dgm_mesh* m, size_t rsize) {
  const size_t pe = (trace_words(m->K, m->pE) * rsize + 255) & ~size_t(255);
  const size_t ph = (trace_words(m->K, m->p) * rsize + 255) & ~size_t(255);
  return kScratchTraceOff + pe + ph;
}

// The workspace laid out as trace buffers and reduction buffers (nothing is allocated;
// nothing needs clearing: the trace buffers are written before they are read and the
// reductions write their results before reading them).
template <typename R>
void noalloc_work(const dgm_mesh* m, void* base, StepWork<R>* ws) {
  unsigned char* b = static_cast<unsigned char*>(base);
  const size_t per = (trace_words(m->K, m->pE) * sizeof(R) + 255) & ~size_t(255);
  ws->partial = reinterpret_cast<double*>(b + kScratchPartialOff);
  ws->res = reinterpret_cast<double*>(b + kScratchResOff);
  ws->TE = reinterpret_cast<R*>(b + kScratchTraceOff);
  ws->TH = reinterpret_cast<R*>(b + kScratchTraceOff + per);
}

}  // namespace

extern "C" {

int dgm_step_noalloc(dgm_mesh* m, int dtype, void* E, void* H, double dt, int64_t nsteps, hipStream_t s) {
  int rc = check_order(m, dtype);
  if (rc) return rc;
  if ((rc = check_constant_material(m, "the allocation-free step"))) return rc;
  if (!E || !H || E == H || nsteps < 0 || !std::isfinite(dt)) return fail(DGM_ERR_ARG, "bad step arguments");
  const size_t rsize = dtype == DGM_F32 ? sizeof(float) : sizeof(double);
  const size_t need = noalloc_bytes(m, rsize);
  if (need > (size_t)DGM_NOALLOC_SCRATCH_BYTES)
    return fail(DGM_ERR_ARG, "mesh too large for the allocation-free step: needs " + std::to_string(need) +
                                 " bytes of workspace, the library holds " +
                                 std::to_string((size_t)DGM_NOALLOC_SCRATCH_BYTES));
  if (nsteps == 0) return DGM_OK;
  void* base = nullptr;
  if ((rc = scratch_address(&base))) return rc;
  if (dtype == DGM_F32) {
    StepWork<float> ws;
    noalloc_work<float>(m, base, &ws);
    return step_impl<float>(m, (float*)E, (float*)H, dt, nsteps, s, ws);
  }
  StepWork<double> ws;
  noalloc_work<double>(m, base, &ws);
  return step_impl<double>(m, (double*)E, (double*)H, dt, nsteps, s, ws);
}

int dgm_energy(dgm_mesh* m, int dtype, const void* E, const void* H, const void* Hn, double dt, double out[2],
               hipStream_t s) {
  // The reductions work at any order; only forming H_next internally needs the
  // order's phase kernel.
  if (!m) return fail(DGM_ERR_ARG, "null mesh");
  if (dtype != DGM_F32 && dtype != DGM_F64) return fail(DGM_ERR_ARG, "dtype must be DGM_F32 or DGM_F64");
  if (m->p < 1) return fail(DGM_ERR_STATE, "order not set (dgm_set_order)");
  if (!E || !H || !out) return fail(DGM_ERR_ARG, "null argument");
  if (!Hn && dt == 0.0) Hn = H;  // Q = W when no step is taken
  int rc;
  if ((!Hn || m->varmat) && (rc = check_order(m, dtype))) return rc;
  if (m->varmat)
    return dtype == DGM_F32 ? energy_var_impl<float>(m, (const float*)E, (const float*)H, (const float*)Hn, dt, out, s)
                            : energy_var_impl<double>(m, (const double*)E, (const double*)H, (const double*)Hn, dt, out, s);
  return dtype == DGM_F32 ? energy_impl<float>(m, (const float*)E, (const float*)H, (const float*)Hn, dt, out, s)
                          : energy_impl<double>(m, (const double*)E, (const double*)H, (const double*)Hn, dt, out, s);
}

int dgm_estimate_dt(dgm_mesh* m, double cfl, int iters, uint64_t seed, double* dt, double* rho_out, hipStream_t s) {
  int rc = check_order(m, DGM_F32);
  if (rc) return rc;
  if (!dt || iters < 1 || !(cfl > 0.0)) return fail(DGM_ERR_ARG, "bad estimate_dt arguments");
  // FP64 vectors where the order is compiled in FP64, FP32 vectors (FP64 dots) above it
  if (m->varmat)
    return m->pE <= DGM_MAX_ORDER_F64 ? estimate_var_impl<double>(m, cfl, iters, seed, dt, rho_out, s)
                                      : estimate_var_impl<float>(m, cfl, iters, seed, dt, rho_out, s);
  return m->pE <= DGM_MAX_ORDER_F64 ? estimate_impl<double>(m, cfl, iters, seed, dt, rho_out, s)
                                   : estimate_impl<float>(m, cfl, iters, seed, dt, rho_out, s);
}

int dgm_apply_curl_dense(dgm_mesh* m, int prec, const float* E, const float* H, float* dE, float* dH, hipStream_t s) {
  int rc = check_order(m, DGM_F32);
  if (rc) return rc;
  if ((rc = check_equal_orders(m, "the dense variant"))) return rc;
  if ((rc = check_constant_material(m, "the dense variant"))) return rc;
  if (prec != DGM_BF16 && prec != DGM_F16) return fail(DGM_ERR_ARG, "precision must be DGM_BF16 or DGM_F16");
  if ((dH && !E) || (dE && !H)) return fail(DGM_ERR_ARG, "output requested without its input");
  if ((dH && (dH == E || dH == H)) || (dE && (dE == E || dE == H))) return fail(DGM_ERR_ARG, "outputs alias inputs");
  DenseOps* d = nullptr;
  if ((rc = dense_ready(m, prec, &d))) return rc;
  if (dH && (rc = dense_rate(m, d, E, dH, 0, s))) return rc;
  if (dE && (rc = dense_rate(m, d, H, dE, 1, s))) return rc;
  return DGM_OK;
}

int dgm_step_dense(dgm_mesh* m, int prec, float* E, float* H, double dt, int64_t nsteps, hipStream_t s) {
  int rc = check_order(m, DGM_F32);
  if (rc) return rc;
  if ((rc = check_equal_orders(m, "the dense variant"))) return rc;
  if ((rc = check_constant_material(m, "the dense variant"))) return rc;
  if (prec != DGM_BF16 && prec != DGM_F16) return fail(DGM_ERR_ARG, "precision must be DGM_BF16 or DGM_F16");
  if (!E || !H || E == H || nsteps < 0 || !std::isfinite(dt)) return fail(DGM_ERR_ARG, "bad step arguments");
  if (nsteps == 0) return DGM_OK;
  DenseOps* d = nullptr;
  if ((rc = dense_ready(m, prec, &d))) return rc;
  if ((rc = convert<float>(m, E, 0, true, s))) return rc;
  if ((rc = convert<float>(m, H, 1, true, s))) return rc;
  for (int64_t it = 0; it < nsteps; ++it) {
    if ((rc = run_dense_phase(m, d, E, H, 0, -dt, s))) return rc;
    if ((rc = run_dense_phase(m, d, H, E, 1, dt, s))) return rc;
  }
  if ((rc = convert<float>(m, E, 0, false, s))) return rc;
  return convert<float>(m, H, 1, false, s);
}

}  // extern "C"

// ---------------------------------------------------------------- batched serving
// Many meshes (slots) advance together: per order, one batched kernel launch per
// leapfrog half step covers every slot of that order, and a chunk of steps for all
// orders is captured once in a HIP graph.  The graph's kernels read the slot
// tables from device memory, so admitting or retiring a slot only rewrites the
// tables; the graph is re-captured only when an order needs a larger grid.
struct dgm_batch {
  struct Slot {
    dgm_mesh* m;
    float* E;
    float* H;
    double dt;
    int64_t left;
    int64_t id;
  };
  int chunk = 0;
  std::vector<Slot> active;
  std::vector<int64_t> finished;
  int64_t next_id = 0;
  BatchSlot* d_slots[DGM_MAX_ORDER_F32 + 1] = {};
  int* d_tile0[DGM_MAX_ORDER_F32 + 1] = {};
  int* d_n[DGM_MAX_ORDER_F32 + 1] = {};
  int cap_slots[DGM_MAX_ORDER_F32 + 1] = {};
  int cap_tiles[DGM_MAX_ORDER_F32 + 1] = {};
  std::vector<BatchSlot> h_slots[DGM_MAX_ORDER_F32 + 1];
  std::vector<int> h_tile0[DGM_MAX_ORDER_F32 + 1];
  int h_n[DGM_MAX_ORDER_F32 + 1] = {};
  hipStream_t cap_stream = nullptr;
  // one capture branch per order (default priority), forked from and joined into cap_stream
  hipStream_t br_stream[DGM_MAX_ORDER_F32 + 1] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[DGM_MAX_ORDER_F32 + 1] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool dirty = true;
  unsigned live_orders = 0;  // orders with active slots in the captured graph
  int streaming = 0;         // nontemporal field accesses (working set of all slots above the cache)
  bool in_flight = false;    // a chunk was launched and not yet waited for
  hipStream_t launch_stream = nullptr;
};

namespace {

int batch_capture(dgm_batch* b) {
  if (b->exec) HIP_TRY(hipGraphExecDestroy(b->exec));
  if (b->graph) HIP_TRY(hipGraphDestroy(b->graph));
  b->exec = nullptr;
  b->graph = nullptr;
  for (int p = 1; p <= DGM_MAX_ORDER_F32; ++p)
    if ((b->live_orders & (1u << p)) && !kBatchF32[p])
      return fail(DGM_ERR_ARG, "batched kernel of order " + std::to_string(p) + " not built");
  if (!b->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  if (!b->fork_ev) HIP_TRY(hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming));
  for (int p = 1; p <= DGM_MAX_ORDER_F32; ++p) {
    if (b->cap_tiles[p] <= 0 || !(b->live_orders & (1u << p))) continue;
    if (!b->br_stream[p]) HIP_TRY(hipStreamCreateWithFlags(&b->br_stream[p], hipStreamNonBlocking));
    if (!b->join_ev[p]) HIP_TRY(hipEventCreateWithFlags(&b->join_ev[p], hipEventDisableTiming));
  }
  // The slots of different orders are independent: each order's chain of half steps is
  // its own branch of the graph (forked from the capture stream, joined back at the end),
  // so the orders' kernels overlap on the device instead of running one after another.
  HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t err = hipEventRecord(b->fork_ev, b->cap_stream);
  for (int p = 1; p <= DGM_MAX_ORDER_F32 && err == hipSuccess; ++p) {
    if (b->cap_tiles[p] <= 0 || !(b->live_orders & (1u << p))) continue;
    err = hipStreamWaitEvent(b->br_stream[p], b->fork_ev, 0);
    for (int sub = 0; sub < b->chunk && err == hipSuccess; ++sub)
      for (int phase = 0; phase < 2 && err == hipSuccess; ++phase) {
        BatchArgs a;
        a.slots = b->d_slots[p];
        a.tile0 = b->d_tile0[p];
        a.nslots = b->d_n[p];
        a.phase = phase;
        a.substep = sub;
        a.blocks = b->cap_tiles[p];
        a.streaming = b->streaming;
        a.stream = b->br_stream[p];
        err = kBatchF32[p](a);
      }
    if (err == hipSuccess) err = hipEventRecord(b->join_ev[p], b->br_stream[p]);
    if (err == hipSuccess) err = hipStreamWaitEvent(b->cap_stream, b->join_ev[p], 0);
  }
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
  if (err != hipSuccess) return fail(DGM_ERR_HIP, std::string("batched launch capture: ") + hipGetErrorString(err));
  if (e2 != hipSuccess) return fail(DGM_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
  b->graph = g;
  HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  b->dirty = false;
  return DGM_OK;
}

}  // namespace

extern "C" {

int dgm_batch_create(int chunk, dgm_batch** out) {
  if (!out || chunk < 1 || chunk > 4096) return fail(DGM_ERR_ARG, "chunk must be in [1, 4096]");
  *out = new dgm_batch();
  (*out)->chunk = chunk;
  return DGM_OK;
}

int dgm_batch_destroy(dgm_batch* b) {
  if (!b) return DGM_OK;
  if (b->in_flight) (void)hipStreamSynchronize(b->launch_stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (int p = 0; p <= DGM_MAX_ORDER_F32; ++p) {
    if (b->br_stream[p]) (void)hipStreamDestroy(b->br_stream[p]);
    if (b->join_ev[p]) (void)hipEventDestroy(b->join_ev[p]);
  }
  if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
  for (int p = 0; p <= DGM_MAX_ORDER_F32; ++p) {
    (void)hipFree(b->d_slots[p]);
    (void)hipFree(b->d_tile0[p]);
    (void)hipFree(b->d_n[p]);
  }
  delete b;
  return DGM_OK;
}

int dgm_batch_add(dgm_batch* b, dgm_mesh* m, float* E, float* H, double dt, int64_t nsteps, hipStream_t s,
                  int64_t* id) {
  if (!b || !E || !H || E == H || nsteps < 0 || !std::isfinite(dt) || !id) return fail(DGM_ERR_ARG, "bad batch slot");
  int rc = check_order(m, DGM_F32);
  if (rc) return rc;
  if ((rc = check_equal_orders(m, "a batch slot"))) return rc;
  if ((rc = check_constant_material(m, "a batch slot"))) return rc;
  for (const auto& q : b->active)
    if (q.m == m) return fail(DGM_ERR_ARG, "mesh handle already has an active slot");
  float *TE, *TH;
  if ((rc = ensure_traces<float>(m, &TE, &TH))) return rc;
  if ((rc = convert<float>(m, E, 0, true, s))) return rc;
  if ((rc = convert<float>(m, H, 1, true, s))) return rc;
  if ((rc = run_trace<float>(m, E, 0, TE, s))) return rc;
  *id = b->next_id++;
  if (nsteps == 0) {
    if ((rc = convert<float>(m, E, 0, false, s))) return rc;
    if ((rc = convert<float>(m, H, 1, false, s))) return rc;
    b->finished.push_back(*id);
    return DGM_OK;
  }
  b->active.push_back({m, E, H, dt, nsteps, *id});
  return DGM_OK;
}

int dgm_batch_num_active(const dgm_batch* b, int64_t* n) {
  if (!b || !n) return fail(DGM_ERR_ARG, "null argument");
  *n = (int64_t)b->active.size();
  return DGM_OK;
}

}  // extern "C"

namespace {

// Whether the next launch re-captures the graph: the set of orders in use, the slot or
// tile capacity of an order or the cache policy no longer matches the captured one.
bool batch_needs_capture(const dgm_batch* b) {
  if (b->dirty || !b->exec) return true;
  int ns[DGM_MAX_ORDER_F32 + 1] = {}, nt[DGM_MAX_ORDER_F32 + 1] = {};
  unsigned live = 0;
  size_t bytes = 0;
  for (const auto& q : b->active) {
    const int p = q.m->p;
    ++ns[p];
    nt[p] += (int)((q.m->K + 63) / 64);
    live |= 1u << p;
    bytes += step_bytes(q.m->K, p, sizeof(float));
  }
  if (live != b->live_orders || (int)(bytes > kStreamingBytes) != b->streaming) return true;
  for (int p = 1; p <= DGM_MAX_ORDER_F32; ++p)
    if (ns[p] > b->cap_slots[p] || nt[p] > b->cap_tiles[p]) return true;
  return false;
}

// Tables, (re-)capture if needed, graph launch and the retirement of finished slots,
// all enqueued on s; the caller waits before the tables or the results are used again.
int batch_launch(dgm_batch* b, hipStream_t s) {
  for (int p = 1; p <= DGM_MAX_ORDER_F32; ++p) {
    b->h_slots[p].clear();
    b->h_tile0[p].assign(1, 0);
  }
  for (const auto& q : b->active) {
    const int p = q.m->p;
    BatchSlot bs;
    bs.E = q.E;
    bs.H = q.H;
    bs.ME = q.m->d_M32[0];
    bs.MH = q.m->d_M32[1];
    bs.nbr = q.m->d_nbr;
    bs.TE = q.m->d_T;
    bs.TH = static_cast<const float*>(q.m->d_T) + trace_words(q.m->K, p);
    bs.K = (int)q.m->K;
    bs.steps_left = (int)std::min<int64_t>(b->chunk, q.left);
    bs.dt = q.dt;
    b->h_slots[p].push_back(bs);
    b->h_tile0[p].push_back(b->h_tile0[p].back() + (int)((q.m->K + 63) / 64));
  }
  for (int p = 1; p <= DGM_MAX_ORDER_F32; ++p) {
    const int ns = (int)b->h_slots[p].size(), nt = b->h_tile0[p].back();
    if (ns > b->cap_slots[p]) {
      const int cap = std::max(ns, 2 * b->cap_slots[p]);
      (void)hipFree(b->d_slots[p]);
      (void)hipFree(b->d_tile0[p]);
      b->d_slots[p] = nullptr;
      b->d_tile0[p] = nullptr;
      HIP_TRY(hipMalloc(&b->d_slots[p], cap * sizeof(BatchSlot)));
      HIP_TRY(hipMalloc(&b->d_tile0[p], (cap + 1) * sizeof(int)));
      if (!b->d_n[p]) HIP_TRY(hipMalloc(&b->d_n[p], sizeof(int)));
      b->cap_slots[p] = cap;
      b->dirty = true;  // table addresses changed
    }
    if (nt > b->cap_tiles[p]) {
      b->cap_tiles[p] = std::max(nt, b->cap_tiles[p] + b->cap_tiles[p] / 2);
      b->dirty = true;
    }
    if (ns > 0) {  // orders without active slots are not in the graph
      b->h_n[p] = ns;
      HIP_TRY(hipMemcpyAsync(b->d_slots[p], b->h_slots[p].data(), ns * sizeof(BatchSlot), hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(b->d_tile0[p], b->h_tile0[p].data(), (ns + 1) * sizeof(int), hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(b->d_n[p], &b->h_n[p], sizeof(int), hipMemcpyHostToDevice, s));
    }
  }
  // the graph covers only the orders that have active slots: re-capture when that set changes
  unsigned live = 0;
  for (int p = 1; p <= DGM_MAX_ORDER_F32; ++p)
    if (!b->h_slots[p].empty()) live |= 1u << p;
  if (live != b->live_orders) {
    b->live_orders = live;
    b->dirty = true;
  }
  size_t bytes = 0;
  for (const auto& q : b->active) bytes += step_bytes(q.m->K, q.m->p, sizeof(float));
  const int streaming = bytes > kStreamingBytes;
  if (streaming != b->streaming) {
    b->streaming = streaming;
    b->dirty = true;
  }
  int rc;
  if (b->dirty && (rc = batch_capture(b))) return rc;
  HIP_TRY(hipGraphLaunch(b->exec, s));
  b->in_flight = true;
  b->launch_stream = s;
  std::vector<dgm_batch::Slot> still;
  for (auto& q : b->active) {
    q.left -= std::min<int64_t>(b->chunk, q.left);
    if (q.left == 0) {
      if ((rc = convert<float>(q.m, q.E, 0, false, s))) return rc;
      if ((rc = convert<float>(q.m, q.H, 1, false, s))) return rc;
      b->finished.push_back(q.id);
    } else {
      still.push_back(q);
    }
  }
  b->active.swap(still);
  return DGM_OK;
}

int batch_wait(dgm_batch* b) {
  if (!b->in_flight) return DGM_OK;
  b->in_flight = false;
  HIP_TRY(hipStreamSynchronize(b->launch_stream));  // host tables are reused by the next launch
  return DGM_OK;
}

}  // namespace

extern "C" {

int dgm_batch_needs_capture(const dgm_batch* b, int* yes) {
  if (!b || !yes) return fail(DGM_ERR_ARG, "null argument");
  *yes = !b->active.empty() && batch_needs_capture(b);
  return DGM_OK;
}

int dgm_batch_launch(dgm_batch* b, hipStream_t s) {
  if (!b) return fail(DGM_ERR_ARG, "null batch");
  if (b->in_flight) return fail(DGM_ERR_STATE, "the previous chunk was not waited for (dgm_batch_wait)");
  if (b->active.empty()) return DGM_OK;
  return batch_launch(b, s);
}

int dgm_batch_wait(dgm_batch* b) {
  if (!b) return fail(DGM_ERR_ARG, "null batch");
  return batch_wait(b);
}

int dgm_batch_advance(dgm_batch* b, hipStream_t s) {
  if (!b) return fail(DGM_ERR_ARG, "null batch");
  if (b->in_flight) return fail(DGM_ERR_STATE, "the previous chunk was not waited for (dgm_batch_wait)");
  if (b->active.empty()) return DGM_OK;
  const int rc = batch_launch(b, s);
  const int rw = batch_wait(b);
  return rc ? rc : rw;
}

int dgm_batch_take_finished(dgm_batch* b, int64_t* ids, int64_t cap, int64_t* n) {
  if (!b || !n || (cap > 0 && !ids)) return fail(DGM_ERR_ARG, "null argument");
  if (b->in_flight) return fail(DGM_ERR_STATE, "results are ready only after dgm_batch_wait");
  const int64_t k = std::min<int64_t>(cap, (int64_t)b->finished.size());
  for (int64_t q = 0; q < k; ++q) ids[q] = b->finished[q];
  b->finished.erase(b->finished.begin(), b->finished.begin() + k);
  *n = k;
  return DGM_OK;
}

}  // extern "C"
