// Descriptors and launch wrappers shared by host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hodbf {

// A factor block (column-major, element (i, k) at f_off + k * lda + i, stored values
// multiplied by scale on load) times the input rows [in_row, in_row + n) of buffer X
// (in_buf = 0) or T (in_buf = 1).
struct Pair {
  int64_t f_off;
  int32_t in_row, n, lda, in_buf;
  float scale;
  int32_t pad;
};

// One output tile of a grouped complex GEMM: m <= 128 rows, the sum over pairs
// [p0, p1) of A_p * in_p.  Its rows are scattered by the row map entries
// [map0, map1) (sorted by start): local row r goes to out_row + r - start of the last
// entry with start <= r, so one tile can hold several stacked blocks that read the
// same input rows.
struct Seg {
  int32_t m, p0, p1, map0, map1, pad0, pad1, pad2;
  Pair first;  // copy of pairs[p0] (set at upload): one dependent load less per tile
};
struct RowMap {
  int32_t start, out_row;
};
constexpr int kTileRows = 64;  // rows of one workgroup tile; leaves hold at most 64 rows
constexpr int kRowClasses = kTileRows / 16;  // tiles of 1..kRowClasses 16-row MFMA tiles
constexpr int kMaxMapEntries = 8;  // row map entries of one tile (the array is padded by as many)


// Device entry-generation job: column-major block of Z, rows r0..r0+m (tree order,
// contiguous), columns cols[c_off .. c_off + n) (tree positions).
struct EntryJob {
  int64_t f_off;
  int32_t r0, m, c_off, n;
};

// Factor storage and arithmetic: complex FP32 (FP32 MFMA); complex BF16 (BF16 MFMA);
// complex FP16 (converted to FP32 on load, FP32 MFMA); complex FP32 with split-BF16
// arithmetic (hi + lo BF16 parts, three BF16 MFMA products, FP32 accumulation).
enum FactorType { FT_C64 = 0, FT_BF16 = 1, FT_F16 = 2, FT_C64_S3 = 3 };

// Grouped GEMM over segs[s0, s0 + ns): OUT(seg rows) = beta * OUT + sum A * in.
// X, T, OUT: complex FP32 RHS-interleaved (element (row, q) at row * R + q).
// The segments of a launch are sorted by row-tile count; cls[c] (c = 0..kRowClasses) is
// the first segment (relative to s0) with more than c row tiles, cls[kRowClasses] = ns.
void launch_grouped(const Seg *segs, const Pair *pairs, const RowMap *rowmap, int64_t s0,
                    int64_t ns, const int64_t *cls, const void *F, int ftype, const float2 *X,
                    const float2 *T, float2 *OUT, int R, int beta, hipStream_t st);

void launch_entries(const EntryJob *jobs, int64_t njobs, const int32_t *cols, const short4 *xyz,
                    const double2 *inv_eps, const double2 *kappa, double kh, double2 k2S,
                    float2 *F32, double2 *F64, hipStream_t st);

// user-order column-major (ld) <-> tree-order RHS-interleaved, with dtype conversion.
// src_c128 / dst_c128 select complex FP64 (true) or FP32 (false) on the user side;
// the tree side is complex FP32 (tree_c128 = false) or FP64.
// tpos[u] = tree position of user index u; perm[i] = user index at tree position i.
void launch_gather(const void *src, bool src_c128, int64_t ld, void *dst, bool dst_c128,
                   const int32_t *tpos, int64_t n, int R, hipStream_t st);
void launch_scatter(const void *src, bool src_c128, void *dst, bool dst_c128, int64_t ld,
                    const int32_t *perm, int64_t n, int R, hipStream_t st);

void launch_plane_wave(const double *dirs_dev, int R, int nx, int ny, int nz, double h,
                       double k0, double2 *b, int64_t ldb, hipStream_t st);

// ---- FP64 Krylov kernels (tree order, RHS-interleaved, complex FP64) ----
void launch_c128_to_c64(const double2 *src, float2 *dst, int64_t count, hipStream_t st);
void launch_c64_to_c128(const float2 *src, double2 *dst, int64_t count, hipStream_t st);
// partial[b][i][q] = sum over rows of block b of conj(V_i(row, q)) * w(row, q), i < nv
void launch_multidot(const double2 *V, int64_t vstride, int nv, const double2 *w, int64_t n,
                     int R, double2 *partial, int nblk, hipStream_t st);
// out[i][q] (+)= sum_b partial[b][i][q]
void launch_reduce_partials(const double2 *partial, int nblk, int nv, int R, double2 *out,
                            int accumulate, hipStream_t st);
int multidot_blocks(int64_t n, int R);
// w -= sum_i V_i * h[i][q]
void launch_vupdate(const double2 *V, int64_t vstride, int nv, const double2 *h, double2 *w,
                    int64_t n, int R, hipStream_t st);
// v = w / hnorm[q] (0 where hnorm is tiny), hnorm given as |.|^2 in re of sq[q]
void launch_normalize(const double2 *w, const double2 *sq, double2 *v, double2 *hcol,
                      int64_t n, int R, const int32_t *active, hipStream_t st);
// x += sum_i Zs_i y_i (Zs complex FP32)
void launch_xupdate(const float2 *Zs, int64_t zstride, int nv, const double2 *y, double2 *x,
                    int64_t n, int R, hipStream_t st);
// out = a - b
void launch_axpby(const double2 *a, const double2 *b, double2 *out, int64_t count, hipStream_t st);
// Column selection on [rows][R]-layout blocks: gather dst[r][k] = src[r][idx[k]] (k < Rd),
// scatter dst[r][idx[k]] = src[r][k] (k < Rs).
template <typename T>
void launch_gather_cols(const T *src, int64_t rows, int Rs, const int32_t *idx, int Rd, T *dst,
                        hipStream_t st);
template <typename T>
void launch_scatter_cols(const T *src, int64_t rows, int Rs, const int32_t *idx, int Rd, T *dst,
                         hipStream_t st);

// Per-column GMRES bookkeeping on the device.  H is stored column by column: column j
// at H + j * (m + 1) * R, entry (i, q) at i * R + q.
struct GmresState {
  double2 *H, *cs, *sn, *g, *y;
  double *bnorm, *est;
  int32_t *jend;    // steps kept in this cycle; -1 while still iterating
  int32_t *active;  // 0 once a column has converged (true residual)
  int m, R;
};
void launch_givens(GmresState s, int j, double tol, hipStream_t st);
void launch_lsq(GmresState s, hipStream_t st);
void launch_cycle_init(GmresState s, const double2 *sq, hipStream_t st);
void launch_mask_cols(double2 *v, const int32_t *active, int64_t n, int R, hipStream_t st);

}  // namespace hodbf
