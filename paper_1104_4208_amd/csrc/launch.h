// Launch arguments shared by the generated per-order phase kernels and the host code.
#pragma once
#include <hip/hip_runtime.h>

// Trace buffer of one field: per element four faces, each holding the two tangential
// traces on the NF face modes (tangent major), each tangent padded to a multiple of four.
// Tiles of 64 elements are contiguous; inside a tile, chunk j (four consecutive
// values of one face) of lane l sits at (j * 64 + l) * 4, so a workgroup stores its
// traces coalesced and a neighbour's chunk is one 16-byte load.
constexpr int trace_face_stride(int NF) { return 2 * ((NF + 3) & ~3); }
constexpr int trace_elem_stride(int NF) { return 4 * trace_face_stride(NF); }

// One 16-byte-aligned chunk of four values (a lane's part of a coalesced store).
__device__ inline void store4(float* p, float a, float b, float c, float d) {
  *reinterpret_cast<float4*>(p) = make_float4(a, b, c, d);
}
__device__ inline void store4(double* p, double a, double b, double c, double d) {
  reinterpret_cast<double2*>(p)[0] = make_double2(a, b);
  reinterpret_cast<double2*>(p)[1] = make_double2(c, d);
}

// Accesses of the phase kernels to the fields (loads of U and of the old V, stores of
// the new V) and stores to the trace buffers.  With ST they carry the nontemporal
// hint; on meshes whose fields and traces exceed the 256 MB last-level cache this
// measured 8 % faster per phase at p = 6, so the host sets it from the working set.
template <bool ST, typename T>
__device__ inline T ldf(const T* p) {
  if constexpr (ST) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool ST, typename T>
__device__ inline void stf(T* p, T v) {
  if constexpr (ST) __builtin_nontemporal_store(v, p);
  else *p = v;
}
template <bool ST>
__device__ inline void store4s(float* p, float a, float b, float c, float d) {
  if constexpr (ST) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 v = {a, b, c, d};
    __builtin_nontemporal_store(v, reinterpret_cast<v4*>(p));
  } else {
    store4(p, a, b, c, d);
  }
}
template <bool ST>
__device__ inline void store4s(double* p, double a, double b, double c, double d) {
  if constexpr (ST) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    const v2 lo = {a, b}, hi = {c, d};
    __builtin_nontemporal_store(lo, reinterpret_cast<v2*>(p));
    __builtin_nontemporal_store(hi, reinterpret_cast<v2*>(p) + 1);
  } else {
    store4(p, a, b, c, d);
  }
}

template <typename R>
struct PhaseArgs {
  const R* U;       // (3,N,K) stored-frame field that is differentiated
  R* V;             // (3,N,K) stored-frame field updated in place: V += sdt * rate
  const R* MU;      // (6,K) symmetric conversion of U into the derivative frame
  const R* MV;      // (6,K) the same for V (traces of the updated V)
  const int* nbr;   // (4,K) neighbour code nb*4 + neighbour's local face, -1 on walls
  const R* Tin;     // traces of U (written by the trace kernel or the previous phase)
  R* Tout;          // traces of the updated V, or nullptr to skip them
  R sdt;            // signed step: -dt (H update) or +dt (E update); -1/+1 for a bare rate
  R wall;           // ghost factor on walls: -1 (E_nb = -E) or +1 (H_nb = H)
  int K;            // number of elements
  int blocks;       // ceil(K / 64)
  int streaming;    // nonzero: nontemporal field and trace-store accesses (ldf, stf, store4s)
  hipStream_t stream;
  // stabilised flux (nullptr HF: central flux).  HF: face unknowns sigma, layout
  // ((k NF + m) 4 + f) K + e, held by each face's owner side; SC: (16,K) the owner's 2x2
  // update matrices; fdt: the step of sigma in the H phase (sigma += fdt C dtau)
  R* HF = nullptr;
  const R* SC = nullptr;
  R fdt = R(0);
  // nonzero: V is only written, V = sdt * rate (central flux, equal orders, no Tout)
  int overwrite = 0;
};

template <typename R>
struct TraceArgs {
  const R* U;       // (3,N,K) stored-frame field
  const R* MU;      // (6,K) its conversion into the derivative frame
  const int* nbr;   // (4,K) neighbour codes: x = 0 / y = 0 faces are stored only across tiles
  R* T;             // traces out (whole tiles)
  int K;
  int blocks;       // ceil(K / 64)
  hipStream_t stream;
};

// Approximate mass inverse of a field with a material linear on every element:
// V = (acc ? V : 0) + s * P X per component, P as in the generated dgm_mass_p{p}.
template <typename R>
struct MassArgs {
  const R* X;       // (3,N,K) input (any frame: P acts on every component alike)
  R* V;             // (3,N,K) output; may not alias X
  const R* mat;     // (4,K) material at the element's vertices, sorted by global id
  R s;              // scale
  int acc;          // nonzero: accumulate into V
  int K;
  int blocks;       // ceil(K / 64); the launch has 3 * blocks workgroups (one per component)
  hipStream_t stream;
};

// One mesh of a batched launch (FP32 fields in the stored frame).
struct BatchSlot {
  const void* E;    // (3,N,K)
  const void* H;    // (3,N,K)
  const void* ME;   // (6,K) conversion of E into the derivative frame
  const void* MH;   // (6,K) conversion of H
  const int* nbr;   // (4,K)
  const void* TE;   // traces of E, kept current by every E update
  const void* TH;   // traces of H, written by every H update
  int K;
  int steps_left;   // sub-steps of the current launch this slot still takes
  double dt;
};

struct BatchArgs {
  const BatchSlot* slots;  // device table, nslots entries
  const int* tile0;        // device prefix sums of tiles, nslots + 1 entries
  const int* nslots;       // device scalar
  int phase;               // 0: H update from E, 1: E update from H
  int substep;             // index of the leapfrog step inside the launch
  int blocks;              // grid size (capacity in tiles)
  int streaming;           // nonzero: nontemporal field and trace-store accesses
  hipStream_t stream;
};
