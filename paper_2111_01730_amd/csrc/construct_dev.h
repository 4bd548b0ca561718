// Device side of the preconditioner construction: elementwise kernels and the device
// engine (construct.h) that runs Algorithm 1 / Algorithm 2 on the grouped-GEMM kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>

namespace hodbf {

class Engine;
struct Tree;

// y += (ar + j ai) x over n complex FP32 values
void launch_axpy_c64(float2 *y, const float2 *x, float ar, float ai, int64_t n, hipStream_t st);
// clear the rows of an N x R multi-vector whose keep flag is 0
void launch_keep_rows(float2 *y, const uint8_t *keep, int64_t rows, int R, hipStream_t st);
// structured random sketch (see Engine::fill_sketch)
void launch_fill_sketch(float2 *x, const int32_t *slot, int64_t rows, int R, int64_t col0, int k,
                        uint64_t seed, hipStream_t st);
// x(r, q) = 1 where q == col[r], else 0
void launch_fill_unit(float2 *x, const int32_t *col, int64_t rows, int R, hipStream_t st);
// out[e k + i] = y(rows[e], q0[e] + i)
void launch_gather_rows(const float2 *y, int R, const int32_t *rows, const int32_t *q0,
                        int64_t nent, int k, float2 *out, hipStream_t st);

// The device engine: multi-vectors in complex FP32 on the GPU (at most max_cols columns
// each), butterfly sets and dense blocks packed into grouped-GEMM programs (forward and
// transposed), everything on one stream.
std::unique_ptr<Engine> make_device_engine(const Tree *t, hipStream_t st, int max_cols);

}  // namespace hodbf
