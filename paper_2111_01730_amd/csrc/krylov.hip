// FP64 Krylov kernels for flexible GMRES: batched multi-dot products with fixed-order
// (deterministic) reductions, vector updates, Givens rotations and the Hessenberg
// least-squares solve, one right-hand side per column of an RHS-interleaved block.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"

namespace hodbf {

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

__global__ void k_c128_to_c64(const double2 *__restrict__ s, float2 *__restrict__ d, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    d[i] = make_float2(float(s[i].x), float(s[i].y));
}
__global__ void k_c64_to_c128(const float2 *__restrict__ s, double2 *__restrict__ d, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    d[i] = make_double2(double(s[i].x), double(s[i].y));
}

static unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return unsigned(b);
}

void launch_c128_to_c64(const double2 *src, float2 *dst, int64_t count, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_c128_to_c64, dim3(grid_for(count)), dim3(256), 0, st, src, dst, count);
}
void launch_c64_to_c128(const float2 *src, double2 *dst, int64_t count, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_c64_to_c128, dim3(grid_for(count)), dim3(256), 0, st, src, dst, count);
}

// Block b handles rows [b*rows_per, (b+1)*rows_per).  Thread t takes column q = t % R
// and row group t / R (R <= 256; larger R loops over column chunks).
__global__ __launch_bounds__(256) void k_multidot(const double2 *__restrict__ V, int64_t vstride,
                                                  int nv, const double2 *__restrict__ w,
                                                  int64_t n, int R, int64_t rows_per,
                                                  double2 *__restrict__ partial) {
  __shared__ double2 red[256];
  const int64_t r0 = int64_t(blockIdx.x) * rows_per;
  int64_t r1 = r0 + rows_per;
  if (r1 > n) r1 = n;
  for (int qc = 0; qc < R; qc += 256) {
    const int Rc = R - qc < 256 ? R - qc : 256;
    const int ng = 256 / Rc;
    const int t = threadIdx.x;
    const int q = qc + t % Rc, g = t / Rc;
    const bool act = g < ng;
    for (int i = 0; i < nv; ++i) {
      double2 acc = make_double2(0.0, 0.0);
      if (act) {
        const double2 *vi = V + int64_t(i) * vstride;
        for (int64_t r = r0 + g; r < r1; r += ng) {
          const int64_t e = r * R + q;
          const double2 p = cmulc(vi[e], w[e]);
          acc.x += p.x;
          acc.y += p.y;
        }
      }
      red[t] = acc;
      __syncthreads();
      if (t < Rc) {
        double2 s = make_double2(0.0, 0.0);
        for (int gg = 0; gg < ng; ++gg) {
          s.x += red[gg * Rc + t].x;
          s.y += red[gg * Rc + t].y;
        }
        partial[(int64_t(blockIdx.x) * nv + i) * R + qc + t] = s;
      }
      __syncthreads();
    }
  }
}

int multidot_blocks(int64_t n, int R) {
  (void)R;
  int64_t b = (n + 63) / 64;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return int(b);
}

void launch_multidot(const double2 *V, int64_t vstride, int nv, const double2 *w, int64_t n,
                     int R, double2 *partial, int nblk, hipStream_t st) {
  const int64_t rows_per = (n + nblk - 1) / nblk;
  hipLaunchKernelGGL(k_multidot, dim3(nblk), dim3(256), 0, st, V, vstride, nv, w, n, R, rows_per,
                     partial);
}

// out[e] (+)= sum over the nblk block partials of element e (e < nv * R).  A workgroup
// owns 16 consecutive elements; its 16 thread groups sum interleaved partials
// (b = g, g + 16, ...) and the 16 group sums are added in group order, so the result
// does not depend on scheduling.
__global__ __launch_bounds__(256) void k_reduce_partials(const double2 *__restrict__ partial,
                                                         int nblk, int nv, int R,
                                                         double2 *__restrict__ out,
                                                         int accumulate) {
  __shared__ double2 red[16][17];
  const int tot = nv * R;
  const int el = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int e = blockIdx.x * 16 + el;
  double2 s = make_double2(0.0, 0.0);
  if (e < tot) {
#pragma unroll 4
    for (int b = g; b < nblk; b += 16) {
      const double2 p = partial[int64_t(b) * tot + e];
      s.x += p.x;
      s.y += p.y;
    }
  }
  red[g][el] = s;
  __syncthreads();
  if (g == 0 && e < tot) {
    double2 t = red[0][el];
    for (int k = 1; k < 16; ++k) {
      t.x += red[k][el].x;
      t.y += red[k][el].y;
    }
    if (accumulate) {
      t.x += out[e].x;
      t.y += out[e].y;
    }
    out[e] = t;
  }
}

void launch_reduce_partials(const double2 *partial, int nblk, int nv, int R, double2 *out,
                            int accumulate, hipStream_t st) {
  const int tot = nv * R;
  hipLaunchKernelGGL(k_reduce_partials, dim3((tot + 15) / 16), dim3(256), 0, st, partial, nblk,
                     nv, R, out, accumulate);
}

__global__ void k_vupdate(const double2 *__restrict__ V, int64_t vstride, int nv,
                          const double2 *__restrict__ h, double2 *__restrict__ w, int64_t n,
                          int R) {
  const int64_t tot = n * R;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int q = int(e % R);
    double2 acc = w[e];
    for (int i = 0; i < nv; ++i) {
      const double2 p = cmul(V[int64_t(i) * vstride + e], h[i * R + q]);
      acc.x -= p.x;
      acc.y -= p.y;
    }
    w[e] = acc;
  }
}

void launch_vupdate(const double2 *V, int64_t vstride, int nv, const double2 *h, double2 *w,
                    int64_t n, int R, hipStream_t st) {
  hipLaunchKernelGGL(k_vupdate, dim3(grid_for(n * R)), dim3(256), 0, st, V, vstride, nv, h, w, n,
                     R);
}

// v = w / ||w|| per column; sq[q].x = ||w_q||^2.  hnorm[q] receives (||w_q||, 0).
__global__ void k_normalize(const double2 *__restrict__ w, const double2 *__restrict__ sq,
                            double2 *__restrict__ v, double2 *__restrict__ hnorm, int64_t n,
                            int R) {
  const int64_t tot = n * R;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int q = int(e % R);
    const double nrm = sqrt(sq[q].x);
    const double inv = nrm > 1e-300 ? 1.0 / nrm : 0.0;
    v[e] = make_double2(w[e].x * inv, w[e].y * inv);
    if (e < R && hnorm) hnorm[q] = make_double2(nrm, 0.0);
  }
}

void launch_normalize(const double2 *w, const double2 *sq, double2 *v, double2 *hcol, int64_t n,
                      int R, const int32_t *active, hipStream_t st) {
  (void)active;
  hipLaunchKernelGGL(k_normalize, dim3(grid_for(n * R)), dim3(256), 0, st, w, sq, v, hcol, n, R);
}

__global__ void k_xupdate(const float2 *__restrict__ Zs, int64_t zstride, int nv,
                          const double2 *__restrict__ y, double2 *__restrict__ x, int64_t n,
                          int R) {
  const int64_t tot = n * R;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int q = int(e % R);
    double2 acc = x[e];
    for (int i = 0; i < nv; ++i) {
      const float2 z = Zs[int64_t(i) * zstride + e];
      const double2 p = cmul(make_double2(z.x, z.y), y[i * R + q]);
      acc.x += p.x;
      acc.y += p.y;
    }
    x[e] = acc;
  }
}

void launch_xupdate(const float2 *Zs, int64_t zstride, int nv, const double2 *y, double2 *x,
                    int64_t n, int R, hipStream_t st) {
  hipLaunchKernelGGL(k_xupdate, dim3(grid_for(n * R)), dim3(256), 0, st, Zs, zstride, nv, y, x,
                     n, R);
}

// out = a - b
__global__ void k_sub(const double2 *__restrict__ a, const double2 *__restrict__ b,
                      double2 *__restrict__ out, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    out[i] = make_double2(a[i].x - b[i].x, a[i].y - b[i].y);
}

void launch_axpby(const double2 *a, const double2 *b, double2 *out, int64_t count, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_sub, dim3(grid_for(count)), dim3(256), 0, st, a, b, out, count);
}

// Column selection on [rows][R]-layout blocks (element (r, q) at r * R + q):
// gather: dst[r][k] = src[r][idx[k]] (k < Rd); scatter: dst[r][idx[k]] = src[r][k].
template <typename T>
__global__ void k_gather_cols(const T *__restrict__ src, int64_t rows, int Rs,
                              const int32_t *__restrict__ idx, int Rd, T *__restrict__ dst) {
  const int64_t tot = rows * Rd;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot;
       e += int64_t(gridDim.x) * blockDim.x)
    dst[e] = src[(e / Rd) * Rs + idx[e % Rd]];
}
template <typename T>
__global__ void k_scatter_cols(const T *__restrict__ src, int64_t rows, int Rs,
                               const int32_t *__restrict__ idx, int Rd, T *__restrict__ dst) {
  const int64_t tot = rows * Rs;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot;
       e += int64_t(gridDim.x) * blockDim.x)
    dst[(e / Rs) * Rd + idx[e % Rs]] = src[e];
}

template <typename T>
void launch_gather_cols(const T *src, int64_t rows, int Rs, const int32_t *idx, int Rd, T *dst,
                        hipStream_t st) {
  if (rows * Rd > 0)
    hipLaunchKernelGGL(k_gather_cols<T>, dim3(grid_for(rows * Rd)), dim3(256), 0, st, src, rows,
                       Rs, idx, Rd, dst);
}
template <typename T>
void launch_scatter_cols(const T *src, int64_t rows, int Rs, const int32_t *idx, int Rd, T *dst,
                         hipStream_t st) {
  if (rows * Rs > 0)
    hipLaunchKernelGGL(k_scatter_cols<T>, dim3(grid_for(rows * Rs)), dim3(256), 0, st, src, rows,
                       Rs, idx, Rd, dst);
}
template void launch_gather_cols<double2>(const double2 *, int64_t, int, const int32_t *, int,
                                          double2 *, hipStream_t);
template void launch_gather_cols<float2>(const float2 *, int64_t, int, const int32_t *, int,
                                         float2 *, hipStream_t);
template void launch_gather_cols<double>(const double *, int64_t, int, const int32_t *, int,
                                         double *, hipStream_t);
template void launch_gather_cols<int32_t>(const int32_t *, int64_t, int, const int32_t *, int,
                                          int32_t *, hipStream_t);
template void launch_scatter_cols<double2>(const double2 *, int64_t, int, const int32_t *, int,
                                           double2 *, hipStream_t);

// ---------------------------------------------------------------------------
// Per-column GMRES bookkeeping (GmresState), one thread per right-hand side.

// Fold the new column j into the QR factorization of the Hessenberg matrix.
__global__ void k_givens(GmresState s, int j, double tol) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= s.R) return;
  if (!s.active[q] || s.jend[q] >= 0) return;
  const int R = s.R;
  double2 *h = s.H + int64_t(j) * (s.m + 1) * R;
  for (int i = 0; i < j; ++i) {
    const double2 c = s.cs[i * R + q], sn = s.sn[i * R + q];
    const double2 a = h[i * R + q], b = h[(i + 1) * R + q];
    const double2 t1 = cmul(c, a), t2 = cmul(sn, b);
    // row 2 of [c s; -conj(s) conj(c)]
    const double2 u1 = cmul(make_double2(-sn.x, sn.y), a);
    const double2 u2 = cmul(make_double2(c.x, -c.y), b);
    h[i * R + q] = make_double2(t1.x + t2.x, t1.y + t2.y);
    h[(i + 1) * R + q] = make_double2(u1.x + u2.x, u1.y + u2.y);
  }
  const double2 a = h[j * R + q], b = h[(j + 1) * R + q];
  const double den = sqrt(a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y);
  double2 c, sn;
  if (den == 0.0) {
    c = make_double2(1.0, 0.0);
    sn = make_double2(0.0, 0.0);
  } else {
    c = make_double2(a.x / den, -a.y / den);   // conj(a) / den
    sn = make_double2(b.x / den, -b.y / den);  // conj(b) / den
  }
  s.cs[j * R + q] = c;
  s.sn[j * R + q] = sn;
  h[j * R + q] = make_double2(den, 0.0);
  h[(j + 1) * R + q] = make_double2(0.0, 0.0);
  const double2 gj = s.g[j * R + q];
  const double2 g1 = cmul(make_double2(-sn.x, sn.y), gj);
  s.g[(j + 1) * R + q] = g1;
  s.g[j * R + q] = cmul(c, gj);
  const double e = sqrt(g1.x * g1.x + g1.y * g1.y);
  s.est[q] = s.bnorm[q] > 0 ? e / s.bnorm[q] : 0.0;
  if (s.est[q] <= tol || j + 1 == s.m || !(e == e)) s.jend[q] = j + 1;
}

// Back-substitution y = R^{-1} g on the rotated Hessenberg matrix, jend steps.
__global__ void k_lsq(GmresState s) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= s.R) return;
  const int R = s.R;
  const int k = s.active[q] ? s.jend[q] : 0;
  for (int i = s.m - 1; i >= k; --i) s.y[i * R + q] = make_double2(0.0, 0.0);
  for (int i = k - 1; i >= 0; --i) {
    double2 acc = s.g[i * R + q];
    for (int l = i + 1; l < k; ++l) {
      const double2 p = cmul(s.H[(int64_t(l) * (s.m + 1) + i) * R + q], s.y[l * R + q]);
      acc.x -= p.x;
      acc.y -= p.y;
    }
    const double2 d = s.H[(int64_t(i) * (s.m + 1) + i) * R + q];
    const double dd = d.x * d.x + d.y * d.y;
    s.y[i * R + q] = dd > 0 ? make_double2((acc.x * d.x + acc.y * d.y) / dd,
                                           (acc.y * d.x - acc.x * d.y) / dd)
                            : make_double2(0.0, 0.0);
  }
}

// Start a cycle: beta = ||r||, v0 = r / beta, g = (beta, 0, ...), jend = -1 for the
// columns still active.  sq[q].x = ||r_q||^2.
__global__ void k_cycle_init(GmresState s, const double2 *__restrict__ sq) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= s.R) return;
  const int R = s.R;
  const double beta = sqrt(sq[q].x);
  for (int i = 0; i <= s.m; ++i) s.g[i * R + q] = make_double2(0.0, 0.0);
  s.g[q] = make_double2(s.active[q] ? beta : 0.0, 0.0);
  s.jend[q] = s.active[q] ? -1 : 0;
}

void launch_givens(GmresState s, int j, double tol, hipStream_t st) {
  hipLaunchKernelGGL(k_givens, dim3((s.R + 63) / 64), dim3(64), 0, st, s, j, tol);
}
void launch_lsq(GmresState s, hipStream_t st) {
  hipLaunchKernelGGL(k_lsq, dim3((s.R + 63) / 64), dim3(64), 0, st, s);
}
void launch_cycle_init(GmresState s, const double2 *sq, hipStream_t st) {
  hipLaunchKernelGGL(k_cycle_init, dim3((s.R + 63) / 64), dim3(64), 0, st, s, sq);
}

// Zero the columns of an RHS-interleaved block whose active flag is 0.
__global__ void k_mask_cols(double2 *__restrict__ v, const int32_t *__restrict__ active,
                            int64_t n, int R) {
  const int64_t tot = n * R;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot;
       e += int64_t(gridDim.x) * blockDim.x)
    if (!active[e % R]) v[e] = make_double2(0.0, 0.0);
}
void launch_mask_cols(double2 *v, const int32_t *active, int64_t n, int R, hipStream_t st) {
  hipLaunchKernelGGL(k_mask_cols, dim3(grid_for(n * R)), dim3(256), 0, st, v, active, n, R);
}

}  // namespace hodbf
