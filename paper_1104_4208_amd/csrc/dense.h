// Dense reference-operator variant (matrix cores): host interface used by dgmax.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

struct DenseOps;

// Assemble the dense operators of order p on the host from the sparse tables and
// upload them as 16-bit values: prec 0 = BF16, 1 = FP16.  Returns 0 or a negative
// DGM_ERR_* code with *err set.
int dense_build(int p, int prec, DenseOps** out, const char** err);
void dense_free(DenseOps* d);
// FP32 scratch the phase needs for the traces of all elements (whole 64-element tiles
// in the trace layout of launch.h).
size_t dense_scratch_floats(const DenseOps* d, int64_t K);
// One phase on stored-frame FP32 fields: V += sdt * rate(U); J is scratch.
hipError_t dense_phase(const DenseOps* d, const float* U, float* V, const float* MU, const int* nbr, float sdt,
                       float wall, int K, float* J, hipStream_t s);
