// Kernels of the preconditioner construction on the device.  Multi-vectors are complex
// FP64, tree order, right-hand sides interleaved (element (i, q) at i R + q): the
// construction multiplies through the multiplicative inverse of the levels below,
// which amplifies rounding by about the condition number, so its products run in FP64
// (factors stored in FP32, as in the applies).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "construct_dev.h"
#include "device.h"
#include "internal.h"
#include "sketch_rng.h"

namespace hodbf {

namespace {

constexpr int kBlock = 256;

unsigned blocks_for(int64_t n) {
  const int64_t b = (n + kBlock - 1) / kBlock;
  return unsigned(b < 65535 * 64 ? b : 65535 * 64);
}

// y += a x over n complex values (grid-stride)
__global__ __launch_bounds__(kBlock) void k_axpy(double2 *__restrict__ y,
                                                 const double2 *__restrict__ x, double ar,
                                                 double ai, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const double2 v = x[i];
    double2 w = y[i];
    w.x += ar * v.x - ai * v.y;
    w.y += ar * v.y + ai * v.x;
    y[i] = w;
  }
}

// rows whose flag is 0 are cleared
__global__ __launch_bounds__(kBlock) void k_keep_rows(double2 *__restrict__ y,
                                                      const uint8_t *__restrict__ keep,
                                                      int64_t rows, int R) {
  const int64_t n = rows * R;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock)
    if (!keep[i / R]) y[i] = make_double2(0.0, 0.0);
}

// x(r, q) = sketch value at global column col0 + q when that column lies in row r's
// slot [slot k, slot k + k), else 0
__global__ __launch_bounds__(kBlock) void k_fill_sketch(double2 *__restrict__ x,
                                                        const int32_t *__restrict__ slot,
                                                        int64_t rows, int R, int64_t col0, int k,
                                                        uint64_t seed) {
  const int64_t n = rows * R;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const int64_t r = i / R;
    const int64_t g = col0 + (i - r * R);
    const int32_t s = slot[r];
    double2 v = make_double2(0.0, 0.0);
    if (s >= 0 && g >= int64_t(s) * k && g < int64_t(s) * k + k) {
      double re, im;
      sketch_parts(seed, uint64_t(r), uint64_t(g), re, im);
      v = make_double2(re, im);
    }
    x[i] = v;
  }
}

__global__ __launch_bounds__(kBlock) void k_fill_unit(double2 *__restrict__ x,
                                                      const int32_t *__restrict__ col,
                                                      int64_t rows, int R) {
  const int64_t n = rows * R;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const int64_t r = i / R;
    x[i] = make_double2(col[r] == int32_t(i - r * R) ? 1.0 : 0.0, 0.0);
  }
}

// out[e k + i] = y(rows[e], q0[e] + i), i < k
__global__ __launch_bounds__(kBlock) void k_gather_rows(const double2 *__restrict__ y, int R,
                                                        const int32_t *__restrict__ rows,
                                                        const int32_t *__restrict__ q0,
                                                        int64_t nent, int k,
                                                        double2 *__restrict__ out) {
  const int64_t n = nent * k;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const int64_t e = i / k;
    const int64_t c = i - e * k;
    out[i] = y[int64_t(rows[e]) * R + q0[e] + c];
  }
}

// ---------------------------------------------------------------------------
// Grouped complex GEMM in FP64 over the descriptors of the applies (device.h): one
// workgroup per (tile, slice of Q right-hand sides); a tile's output rows (at most
// kTileRows) are the sum over its pairs of the FP32-stored factor block (times the
// pair's scale) and its input rows, accumulated in FP64; rows are scattered through the
// tile's row map (beta 0 stores, beta 1 adds: every output element has one owner).
// Factor and input chunks of kK columns pass through LDS.  Q = 32 for wide
// multi-vectors (the construction), 16 or 8 for at most 16 or 8 columns (the solver's
// last columns), so narrow products do not pay for 32.
constexpr int kK = 16;  // inner-dimension chunk

template <int Q>
__global__ __launch_bounds__(kBlock) void k_grouped_f64(
    const Seg *__restrict__ segs, const Pair *__restrict__ pairs, const RowMap *__restrict__ rowmap,
    const float2 *__restrict__ F, const double2 *__restrict__ X, const double2 *__restrict__ T,
    double2 *__restrict__ OUT, int R, int beta, int nsl) {
  constexpr int kPerThread = kTileRows * Q / kBlock;  // outputs per thread (8 or 2)
  static_assert(kPerThread * kBlock == kTileRows * Q, "tile not divisible");
  __shared__ double2 As[kK][kTileRows];
  __shared__ double2 Xs[kK][Q];
  const int tid = threadIdx.x;
  const int seg = blockIdx.x / nsl;
  const int q0 = (blockIdx.x % nsl) * Q;
  const Seg sg = segs[seg];
  const int row = tid % kTileRows;   // output row of this thread
  const int qg = tid / kTileRows;    // its group of kPerThread columns
  double2 acc[kPerThread];
#pragma unroll
  for (int c = 0; c < kPerThread; ++c) acc[c] = make_double2(0.0, 0.0);
  for (int p = sg.p0; p < sg.p1; ++p) {
    const Pair pr = pairs[p];
    const double2 *in = pr.in_buf ? T : X;
    for (int k0 = 0; k0 < pr.n; k0 += kK) {
      // factor chunk: kK columns of the tile's rows
      for (int e = tid; e < kK * kTileRows; e += kBlock) {
        const int kk = e / kTileRows, i = e % kTileRows;
        double2 a = make_double2(0.0, 0.0);
        if (i < sg.m && k0 + kk < pr.n) {
          const float2 f = F[pr.f_off + int64_t(k0 + kk) * pr.lda + i];
          a = make_double2(double(f.x) * pr.scale, double(f.y) * pr.scale);
        }
        As[kk][i] = a;
      }
      // input chunk: kK rows of the pair's input, Q columns
      for (int e = tid; e < kK * Q; e += kBlock) {
        const int kk = e / Q, q = e % Q;
        double2 v = make_double2(0.0, 0.0);
        if (k0 + kk < pr.n && q0 + q < R) v = in[int64_t(pr.in_row + k0 + kk) * R + q0 + q];
        Xs[kk][q] = v;
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < kK; ++kk) {
        const double2 a = As[kk][row];
#pragma unroll
        for (int c = 0; c < kPerThread; ++c) {
          const double2 v = Xs[kk][qg * kPerThread + c];
          acc[c].x += a.x * v.x - a.y * v.y;
          acc[c].y += a.x * v.y + a.y * v.x;
        }
      }
      __syncthreads();
    }
  }
  if (row >= sg.m) return;
  int base = 0;
  for (int e = sg.map0; e < sg.map1; ++e)
    if (rowmap[e].start <= row) base = rowmap[e].out_row - rowmap[e].start;
  double2 *o = OUT + int64_t(base + row) * R;
#pragma unroll
  for (int c = 0; c < kPerThread; ++c) {
    const int q = q0 + qg * kPerThread + c;
    if (q >= R) continue;
    if (beta) {
      o[q].x += acc[c].x;
      o[q].y += acc[c].y;
    } else {
      o[q] = acc[c];
    }
  }
}

}  // namespace

void launch_axpy_c128(double2 *y, const double2 *x, double ar, double ai, int64_t n,
                      hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_axpy, dim3(blocks_for(n)), dim3(kBlock), 0, st, y, x, ar, ai, n);
}

void launch_keep_rows_c128(double2 *y, const uint8_t *keep, int64_t rows, int R, hipStream_t st) {
  if (rows * R <= 0) return;
  hipLaunchKernelGGL(k_keep_rows, dim3(blocks_for(rows * R)), dim3(kBlock), 0, st, y, keep, rows, R);
}

void launch_fill_sketch_c128(double2 *x, const int32_t *slot, int64_t rows, int R, int64_t col0,
                             int k, uint64_t seed, hipStream_t st) {
  if (rows * R <= 0) return;
  hipLaunchKernelGGL(k_fill_sketch, dim3(blocks_for(rows * R)), dim3(kBlock), 0, st, x, slot, rows,
                     R, col0, k, seed);
}

void launch_fill_unit_c128(double2 *x, const int32_t *col, int64_t rows, int R, hipStream_t st) {
  if (rows * R <= 0) return;
  hipLaunchKernelGGL(k_fill_unit, dim3(blocks_for(rows * R)), dim3(kBlock), 0, st, x, col, rows, R);
}

void launch_gather_rows_c128(const double2 *y, int R, const int32_t *rows, const int32_t *q0,
                             int64_t nent, int k, double2 *out, hipStream_t st) {
  if (nent * k <= 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3(blocks_for(nent * k)), dim3(kBlock), 0, st, y, R, rows, q0,
                     nent, k, out);
}

void launch_grouped_f64(const Seg *segs, const Pair *pairs, const RowMap *rowmap, int64_t s0,
                        int64_t ns, const float2 *F, const double2 *X, const double2 *T,
                        double2 *OUT, int R, int beta, hipStream_t st) {
  if (ns <= 0 || R <= 0) return;
  const int q = R <= 8 ? 8 : (R <= 16 ? 16 : 32);
  const int nsl = (R + q - 1) / q;
  const int64_t items = ns * nsl;
  if (items > (int64_t(1) << 31) - 1) fail(HODBF_E_ARG, "construction launch too large");
  if (q == 8)
    hipLaunchKernelGGL(k_grouped_f64<8>, dim3(unsigned(items)), dim3(kBlock), 0, st, segs + s0,
                       pairs, rowmap, F, X, T, OUT, R, beta, nsl);
  else if (q == 16)
    hipLaunchKernelGGL(k_grouped_f64<16>, dim3(unsigned(items)), dim3(kBlock), 0, st, segs + s0,
                       pairs, rowmap, F, X, T, OUT, R, beta, nsl);
  else
    hipLaunchKernelGGL(k_grouped_f64<32>, dim3(unsigned(items)), dim3(kBlock), 0, st, segs + s0,
                       pairs, rowmap, F, X, T, OUT, R, beta, nsl);
}

}  // namespace hodbf
