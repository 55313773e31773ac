// Dense reference-operator variant of one leapfrog phase on the matrix cores.
//
// The same operator as the sparse phase kernels, written as two dense matrices
// that act on a tile of 64 elements at once (one element per GEMM column), with
// 16-bit operands (BF16 or FP16) and FP32 accumulation on
// v_mfma_f32_32x32x16_{bf16,f16}:
//   AT   [8 NF x 3N]        tangential traces on the four faces  tau_{f,k} = T_f (g_{f,k} . w)
//   AU   [3N x (3N + 8NF)]  curl in the derivative frame plus the lifted jumps
// where w = M S is the element's field in the derivative frame.  Section 3.2
// evaluates these operators with O(N) recurrences; this variant applies them
// as the O(N^2) matrix-vector products the paper avoids, batched over elements
// so that they run on the matrix cores.  The field update itself stays FP32.
//
// Two kernels per phase: dense_trace writes every element's own traces (FP32) to a
// scratch buffer J in the trace layout of the sparse path; dense_update forms the
// jumps (neighbour minus own, read from J) and adds sdt * (A_U [w; jumps]) to the
// updated field.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "dense.h"
#include "launch.h"
#include "generated/tables.inc"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kTile = 64;      // elements per workgroup (two 32-wide MFMA column tiles)
constexpr int kThreads = 1024; // sixteen waves (one WG per CU: the waves hide each other's L2 latency)
constexpr int kPad = 8;        // extra 16-bit entries per LDS row

template <typename T> struct Vec8;
template <> struct Vec8<__bf16> { typedef bf16x8 type; };
template <> struct Vec8<_Float16> { typedef f16x8 type; };

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mfma(f16x8 a, f16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

__host__ __device__ constexpr int rup(int x, int m) { return (x + m - 1) / m * m; }

// Tile of 64 elements: rows rt*32.. of A (row-major, lda = KP) times the LDS
// operand Bs (element-major rows of stride KP + kPad).  acc0 / acc1 receive the
// 32 x 32 blocks of element columns 0..31 / 32..63; entry i of this lane is row
// rt*32 + 8*(i/4) + 4*(lane/32) + i%4, column lane%32.
template <typename T>
__device__ __forceinline__ void gemm_acc(const T* __restrict__ A, int KP, const T* Bs, int rt, f32x16& acc0,
                                         f32x16& acc1) {
  typedef typename Vec8<T>::type V8;
  const int l = threadIdx.x & 63;
  const int half = l >> 5, r = l & 31;
  acc0 = f32x16{};
  acc1 = f32x16{};
  // the operator is stored in fragment order (frag_order): the 64 lanes' fragments of
  // one row tile and k-step are one contiguous 1 KB block
  const V8* af = reinterpret_cast<const V8*>(A) + (size_t)rt * (KP / 16) * 64 + l;
  const T* b0 = Bs + (size_t)r * (KP + kPad) + half * 8;
  const T* b1 = Bs + (size_t)(32 + r) * (KP + kPad) + half * 8;
  // operator fragments are fetched (from L2) three k-steps ahead
  const int last = KP / 16 - 1;
  V8 a0 = af[0];
  V8 a1 = af[(1 < last ? 1 : last) * 64];
  V8 a2 = af[(2 < last ? 2 : last) * 64];
#pragma unroll 4
  for (int ks = 0; ks < KP; ks += 16) {
    const int s3 = ks / 16 + 3;
    const V8 a3 = af[(s3 < last ? s3 : last) * 64];
    const V8 x0 = *reinterpret_cast<const V8*>(b0 + ks);
    const V8 x1 = *reinterpret_cast<const V8*>(b1 + ks);
    acc0 = mfma(a0, x0, acc0);
    acc1 = mfma(a0, x1, acc1);
    a0 = a1;
    a1 = a2;
    a2 = a3;
  }
}

__device__ __forceinline__ int acc_row(int rt, int i) { return rt * 32 + 8 * (i >> 2) + 4 * ((threadIdx.x & 63) >> 5) + (i & 3); }

// Fill one LDS row block with w = scale * M S of the given elements (16-bit).
template <typename T>
__device__ void fill_w(T* Bs, int KP, const float* __restrict__ U, const float* __restrict__ MU, int N, int K,
                       const int* src, const float* scale, int col0) {
  const size_t Ks = (size_t)K;
  // thread: element j, modes a0, a0 + 4, ...; the metric is read once and eight
  // modes' loads are in flight together
  const int j = threadIdx.x % kTile, a0 = threadIdx.x / kTile;
  const int e = src[j];
  const int es = e >= 0 ? e : 0;
  const float c = e >= 0 ? scale[j] : 0.f;
  const float m00 = c * MU[0 * Ks + es], m01 = c * MU[1 * Ks + es], m02 = c * MU[2 * Ks + es];
  const float m11 = c * MU[3 * Ks + es], m12 = c * MU[4 * Ks + es], m22 = c * MU[5 * Ks + es];
  T* row = Bs + (size_t)j * (KP + kPad) + col0;
#pragma unroll 8
  for (int a = a0; a < N; a += kThreads / kTile) {
    const float s0 = U[(size_t)a * Ks + es], s1 = U[(size_t)(N + a) * Ks + es], s2 = U[(size_t)(2 * N + a) * Ks + es];
    row[a] = (T)(m00 * s0 + m01 * s1 + m02 * s2);
    row[N + a] = (T)(m01 * s0 + m11 * s1 + m12 * s2);
    row[2 * N + a] = (T)(m02 * s0 + m12 * s1 + m22 * s2);
  }
}

// Own traces of a tile: J[row][e] = (AT w_e)[row], rows (f*2 + k)*NF + m, as one GEMM
// of the trace table against the tile's field in the derivative frame.
template <typename T>
__global__ void __launch_bounds__(kThreads) dense_trace_kernel(const float* __restrict__ U, const float* __restrict__ MU,
                                                               int K, int N, int NF, int KP,
                                                               const T* __restrict__ AT, float* __restrict__ J) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* Bs = reinterpret_cast<T*>(smem);
  __shared__ int src[kTile];
  __shared__ float scl[kTile];
  const int wave = threadIdx.x >> 6;
  const int e0 = blockIdx.x * kTile;
  const size_t Ks = (size_t)K;
  if (threadIdx.x < kTile) {
    const int e = e0 + threadIdx.x;
    src[threadIdx.x] = e < K ? e : -1;
    scl[threadIdx.x] = 1.f;
  }
  for (int idx = threadIdx.x; idx < kTile * (KP + kPad - 3 * N); idx += kThreads) {
    const int j = idx / (KP + kPad - 3 * N), c = 3 * N + idx % (KP + kPad - 3 * N);
    Bs[(size_t)j * (KP + kPad) + c] = (T)0.f;
  }
  __syncthreads();
  fill_w<T>(Bs, KP, U, MU, N, K, src, scl, 0);
  __syncthreads();
  const int M1 = 8 * NF;
  // traces go to the tile-blocked, quad-interleaved layout of the sparse path
  // (launch.h): value c = k * NFP + m of face f, lane l at ((f FQ + c/4) 64 + l) 4 + c%4
  const int r = threadIdx.x & 31;
  const int NFP = trace_face_stride(NF) / 2, FQ = NFP / 2;
  float* Jt = J + (size_t)blockIdx.x * kTile * trace_elem_stride(NF);
  for (int rt = wave; rt * 32 < M1; rt += kThreads / 64) {
    f32x16 acc0, acc1;
    gemm_acc<T>(AT, KP, Bs, rt, acc0, acc1);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = acc_row(rt, i);
      if (row < M1) {
        const int f = row / (2 * NF), km = row - f * 2 * NF, k = km >= NF, c = km + k * (NFP - NF);
        const int off = ((f * FQ + (c >> 2)) * kTile) * 4 + (c & 3);
        Jt[off + r * 4] = acc0[i];
        Jt[off + (32 + r) * 4] = acc1[i];
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) dense_update_kernel(const float* __restrict__ U, float* __restrict__ V,
                                                                const float* __restrict__ MU,
                                                                const int* __restrict__ nbr,
                                                                const float* __restrict__ J, float sdt, float wall,
                                                                int K, int N, int NF, int KP,
                                                                const T* __restrict__ AU) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* Bs = reinterpret_cast<T*>(smem);
  __shared__ int src[kTile];
  __shared__ float scl[kTile];
  const int wave = threadIdx.x >> 6;
  const int e0 = blockIdx.x * kTile;
  const size_t Ks = (size_t)K;
  if (threadIdx.x < kTile) {
    const int e = e0 + threadIdx.x;
    src[threadIdx.x] = e < K ? e : -1;
    scl[threadIdx.x] = 1.f;
  }
  const int c0 = 3 * N + 8 * NF;
  for (int idx = threadIdx.x; idx < kTile * (KP + kPad - c0); idx += kThreads) {
    const int j = idx / (KP + kPad - c0), c = c0 + idx % (KP + kPad - c0);
    Bs[(size_t)j * (KP + kPad) + c] = (T)0.f;
  }
  __syncthreads();
  fill_w<T>(Bs, KP, U, MU, N, K, src, scl, 0);
  // jumps of the tangential traces, neighbour minus own ((wall - 1) times own on walls),
  // from the traces of all elements in the tile-blocked layout: per lane one 16-byte
  // load of the own and one of the neighbour's chunk (four face modes of one tangent)
  {
    const int j = threadIdx.x % kTile, q0 = threadIdx.x / kTile;
    const int e = e0 + j;
    const int es = e < K ? e : K - 1;
    const int NFP = trace_face_stride(NF) / 2, FQ = NFP / 2, ES = trace_elem_stride(NF);
    const float* own = J + (size_t)(es >> 6) * kTile * ES + (size_t)(es & 63) * 4;
    T* row = Bs + (size_t)j * (KP + kPad) + 3 * N;
#pragma unroll 4
    for (int q = q0; q < 4 * FQ; q += kThreads / kTile) {
      const int f = q / FQ, c = 4 * (q - f * FQ), k = c >= NFP, m = c - k * NFP;
      const int code = nbr[(size_t)f * Ks + es];
      const int nb = code < 0 ? es : code >> 2, gf = code < 0 ? f : code & 3;
      const float4 o = *reinterpret_cast<const float4*>(own + (size_t)q * kTile * 4);
      const float4 t = *reinterpret_cast<const float4*>(J + (size_t)(nb >> 6) * kTile * ES +
                                                        ((size_t)(gf * FQ + (q - f * FQ)) * kTile + (nb & 63)) * 4);
      const float cw = code < 0 ? wall - 1.f : -1.f, cn = code < 0 ? 0.f : 1.f;
      const float v[4] = {cn * t.x + cw * o.x, cn * t.y + cw * o.y, cn * t.z + cw * o.z, cn * t.w + cw * o.w};
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (m + i < NF) row[(f * 2 + k) * NF + m + i] = (T)(e < K ? v[i] : 0.f);
    }
  }
  __syncthreads();
  const int M3 = 3 * N;
  const int r = threadIdx.x & 31;
  for (int rt = wave; rt * 32 < M3; rt += kThreads / 64) {
    f32x16 acc0, acc1;
    gemm_acc<T>(AU, KP, Bs, rt, acc0, acc1);
    // all old values of the block first, then the updates (no load waits behind a store)
    float old0[16], old1[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = acc_row(rt, i);
      old0[i] = (row < M3 && e0 + r < K) ? V[(size_t)row * Ks + e0 + r] : 0.f;
      old1[i] = (row < M3 && e0 + 32 + r < K) ? V[(size_t)row * Ks + e0 + 32 + r] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = acc_row(rt, i);
      if (row < M3 && e0 + r < K) V[(size_t)row * Ks + e0 + r] = old0[i] + sdt * acc0[i];
      if (row < M3 && e0 + 32 + r < K) V[(size_t)row * Ks + e0 + 32 + r] = old1[i] + sdt * acc1[i];
    }
  }
}

uint16_t to_bf16(double x) {
  const float f = (float)x;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t rounding = 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)((u + rounding) >> 16);
}

uint16_t to_f16(double x) {
  const _Float16 h = (_Float16)(float)x;
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}

}  // namespace

struct DenseOps {
  int p = 0, prec = 0, N = 0, NF = 0, KP1 = 0, KP2 = 0;
  void* AT = nullptr;
  void* AU = nullptr;
};

int dense_build(int p, int prec, DenseOps** out, const char** err) {
  *out = nullptr;
  if (p < 1 || p > (int)(sizeof(kTables) / sizeof(kTables[0])) - 1 || kTables[p].N == 0) {
    *err = "order out of range for the dense variant";
    return -1;
  }
  const OrderTables& t = kTables[p];
  const int N = t.N, NF = t.NF;
  const int KP1 = rup(3 * N, 16), KP2 = rup(3 * N + 8 * NF, 16);
  const int M1P = rup(8 * NF, 32), M3P = rup(3 * N, 32);
  std::vector<double> AT((size_t)M1P * KP1, 0.0), AU((size_t)M3P * KP2, 0.0);
  for (int f = 0; f < 4; ++f)
    for (int q = 0; q < t.nT[f]; ++q) {
      const SparseEntry& s = t.T[f][q];
      for (int k = 0; k < 2; ++k)
        for (int c = 0; c < 3; ++c) {
          AT[(size_t)((f * 2 + k) * NF + s.r) * KP1 + c * N + s.c] += t.g[f][k][c] * s.v;
        }
      for (int k = 0; k < 3; ++k)
        for (int sc = 0; sc < 2; ++sc)
          AU[(size_t)(k * N + s.c) * KP2 + 3 * N + (f * 2 + sc) * NF + s.r] += t.Lp[f][k][sc] * s.v;
    }
  static const int cyc[3][2] = {{1, 2}, {2, 0}, {0, 1}};
  for (int k = 0; k < 3; ++k) {
    const int i = cyc[k][0], j = cyc[k][1];
    for (int q = 0; q < t.nD[i]; ++q) {  // + D_i w_j
      const SparseEntry& s = t.D[i][q];
      AU[(size_t)(k * N + s.r) * KP2 + j * N + s.c] += s.v;
    }
    for (int q = 0; q < t.nD[j]; ++q) {  // - D_j w_i
      const SparseEntry& s = t.D[j][q];
      AU[(size_t)(k * N + s.r) * KP2 + i * N + s.c] -= s.v;
    }
  }
  // fragment order: block (row tile rt, k-step s) holds, for lane l, the 8 values of
  // row rt*32 + l%32 at columns s*16 + (l/32)*8 .. +7 (the MFMA A-operand layout)
  auto frag_order = [](const std::vector<double>& a, int rows, int KP) {
    std::vector<double> o(a.size());
    size_t q = 0;
    for (int rt = 0; rt < rows / 32; ++rt)
      for (int s = 0; s < KP / 16; ++s)
        for (int l = 0; l < 64; ++l)
          for (int i = 0; i < 8; ++i) o[q++] = a[(size_t)(rt * 32 + l % 32) * KP + s * 16 + (l / 32) * 8 + i];
    return o;
  };
  auto conv = [&](const std::vector<double>& rowmajor, int rows, int KP, void** dst) -> int {
    const std::vector<double> src = frag_order(rowmajor, rows, KP);
    std::vector<uint16_t> h(src.size());
    for (size_t q = 0; q < src.size(); ++q) h[q] = prec == 0 ? to_bf16(src[q]) : to_f16(src[q]);
    if (hipMalloc(dst, h.size() * 2) != hipSuccess) return -5;
    if (hipMemcpy(*dst, h.data(), h.size() * 2, hipMemcpyHostToDevice) != hipSuccess) return -6;
    return 0;
  };
  auto* d = new DenseOps();
  d->p = p;
  d->prec = prec;
  d->N = N;
  d->NF = NF;
  d->KP1 = KP1;
  d->KP2 = KP2;
  int rc = conv(AT, M1P, KP1, &d->AT);
  if (!rc) rc = conv(AU, M3P, KP2, &d->AU);
  if (rc) {
    dense_free(d);
    *err = "device allocation for the dense operators failed";
    return rc;
  }
  *out = d;
  return 0;
}

void dense_free(DenseOps* d) {
  if (!d) return;
  (void)hipFree(d->AT);
  (void)hipFree(d->AU);
  delete d;
}

size_t dense_scratch_floats(const DenseOps* d, int64_t K) {
  return (size_t)((K + kTile - 1) / kTile) * kTile * trace_elem_stride(d->NF);
}

template <typename T>
static hipError_t dense_phase_t(const DenseOps* d, const float* U, float* V, const float* MU, const int* nbr,
                                float sdt, float wall, int K, float* J, hipStream_t s) {
  const int blocks = (K + kTile - 1) / kTile;
  const size_t lds1 = (size_t)kTile * (d->KP1 + kPad) * sizeof(T);
  const size_t lds2 = (size_t)kTile * (d->KP2 + kPad) * sizeof(T);
  hipError_t e = hipFuncSetAttribute((const void*)dense_trace_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds1);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)dense_update_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dense_trace_kernel<T>, dim3(blocks), dim3(kThreads), lds1, s, U, MU, K, d->N, d->NF, d->KP1,
                     (const T*)d->AT, J);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dense_update_kernel<T>, dim3(blocks), dim3(kThreads), lds2, s, U, V, MU, nbr, (const float*)J, sdt,
                     wall, K, d->N, d->NF, d->KP2, (const T*)d->AU);
  return hipGetLastError();
}

hipError_t dense_phase(const DenseOps* d, const float* U, float* V, const float* MU, const int* nbr, float sdt,
                       float wall, int K, float* J, hipStream_t s) {
  return d->prec == 0 ? dense_phase_t<__bf16>(d, U, V, MU, nbr, sdt, wall, K, J, s)
                      : dense_phase_t<_Float16>(d, U, V, MU, nbr, sdt, wall, K, J, s);
}
