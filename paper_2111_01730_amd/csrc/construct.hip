// Elementwise kernels of the preconditioner construction on the device: multi-vectors
// are complex FP32, tree order, right-hand sides interleaved (element (i, q) at i R + q).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "construct_dev.h"
#include "sketch_rng.h"

namespace hodbf {

namespace {

constexpr int kBlock = 256;

unsigned blocks_for(int64_t n) {
  const int64_t b = (n + kBlock - 1) / kBlock;
  return unsigned(b < 65535 * 64 ? b : 65535 * 64);
}

// y += a x over n complex values (grid-stride)
__global__ __launch_bounds__(kBlock) void k_axpy(float2 *__restrict__ y,
                                                 const float2 *__restrict__ x, float ar,
                                                 float ai, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const float2 v = x[i];
    float2 w = y[i];
    w.x += ar * v.x - ai * v.y;
    w.y += ar * v.y + ai * v.x;
    y[i] = w;
  }
}

// rows whose flag is 0 are cleared
__global__ __launch_bounds__(kBlock) void k_keep_rows(float2 *__restrict__ y,
                                                      const uint8_t *__restrict__ keep,
                                                      int64_t rows, int R) {
  const int64_t n = rows * R;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock)
    if (!keep[i / R]) y[i] = make_float2(0.f, 0.f);
}

// x(r, q) = sketch value at global column col0 + q when that column lies in row r's
// slot [slot k, slot k + k), else 0
__global__ __launch_bounds__(kBlock) void k_fill_sketch(float2 *__restrict__ x,
                                                        const int32_t *__restrict__ slot,
                                                        int64_t rows, int R, int64_t col0, int k,
                                                        uint64_t seed) {
  const int64_t n = rows * R;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const int64_t r = i / R;
    const int64_t g = col0 + (i - r * R);
    const int32_t s = slot[r];
    float2 v = make_float2(0.f, 0.f);
    if (s >= 0 && g >= int64_t(s) * k && g < int64_t(s) * k + k) {
      double re, im;
      sketch_parts(seed, uint64_t(r), uint64_t(g), re, im);
      v = make_float2(float(re), float(im));
    }
    x[i] = v;
  }
}

__global__ __launch_bounds__(kBlock) void k_fill_unit(float2 *__restrict__ x,
                                                      const int32_t *__restrict__ col,
                                                      int64_t rows, int R) {
  const int64_t n = rows * R;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const int64_t r = i / R;
    x[i] = make_float2(col[r] == int32_t(i - r * R) ? 1.f : 0.f, 0.f);
  }
}

// out[e k + i] = y(rows[e], q0[e] + i), i < k
__global__ __launch_bounds__(kBlock) void k_gather_rows(const float2 *__restrict__ y, int R,
                                                        const int32_t *__restrict__ rows,
                                                        const int32_t *__restrict__ q0,
                                                        int64_t nent, int k,
                                                        float2 *__restrict__ out) {
  const int64_t n = nent * k;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const int64_t e = i / k;
    const int64_t c = i - e * k;
    out[i] = y[int64_t(rows[e]) * R + q0[e] + c];
  }
}

}  // namespace

void launch_axpy_c64(float2 *y, const float2 *x, float ar, float ai, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_axpy, dim3(blocks_for(n)), dim3(kBlock), 0, st, y, x, ar, ai, n);
}

void launch_keep_rows(float2 *y, const uint8_t *keep, int64_t rows, int R, hipStream_t st) {
  if (rows * R <= 0) return;
  hipLaunchKernelGGL(k_keep_rows, dim3(blocks_for(rows * R)), dim3(kBlock), 0, st, y, keep, rows, R);
}

void launch_fill_sketch(float2 *x, const int32_t *slot, int64_t rows, int R, int64_t col0, int k,
                        uint64_t seed, hipStream_t st) {
  if (rows * R <= 0) return;
  hipLaunchKernelGGL(k_fill_sketch, dim3(blocks_for(rows * R)), dim3(kBlock), 0, st, x, slot, rows,
                     R, col0, k, seed);
}

void launch_fill_unit(float2 *x, const int32_t *col, int64_t rows, int R, hipStream_t st) {
  if (rows * R <= 0) return;
  hipLaunchKernelGGL(k_fill_unit, dim3(blocks_for(rows * R)), dim3(kBlock), 0, st, x, col, rows, R);
}

void launch_gather_rows(const float2 *y, int R, const int32_t *rows, const int32_t *q0,
                        int64_t nent, int k, float2 *out, hipStream_t st) {
  if (nent * k <= 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3(blocks_for(nent * k)), dim3(kBlock), 0, st, y, R, rows, q0,
                     nent, k, out);
}

}  // namespace hodbf
