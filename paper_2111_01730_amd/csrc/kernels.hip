// HIP kernels for gfx950: entry generation, permutation, and the grouped complex GEMM
// that applies every butterfly factor stage and the leaf / outer blocks.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <type_traits>

#include "device.h"

namespace hodbf {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Entry generation (K1).  Z(m, n) = delta_mn / eps_m - K(d_mn) kappa_n with
// K(d) = (kh)^2 / (4 pi |d|) exp(-j kh |d|), K(0) = k^2 S(a) (Section II, voxel
// collocation).  Distances come from exact integer offsets; the phase is evaluated
// in FP64 so that large k|R| keeps full accuracy, then rounded to the output type.
__global__ __launch_bounds__(256) void k_entries(const EntryJob *__restrict__ jobs,
                                                 const int32_t *__restrict__ cols,
                                                 const short4 *__restrict__ xyz,
                                                 const double2 *__restrict__ inv_eps,
                                                 const double2 *__restrict__ kappa, double kh,
                                                 double2 k2S, float2 *__restrict__ F32,
                                                 double2 *__restrict__ F64) {
  const EntryJob jb = jobs[blockIdx.x];
  const int64_t total = int64_t(jb.m) * jb.n;
  const double c0 = kh * kh * (1.0 / (4.0 * M_PI));
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int i = int(e % jb.m);
    const int k = int(e / jb.m);
    const int32_t row = jb.r0 + i;
    const int32_t col = cols[jb.c_off + k];
    const short4 a = xyz[row], b = xyz[col];
    const int dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    const int d2 = dx * dx + dy * dy + dz * dz;
    const double2 kap = kappa[col];
    double2 z;
    if (d2 == 0) {
      const double2 ie = inv_eps[row];
      z.x = ie.x - (k2S.x * kap.x - k2S.y * kap.y);
      z.y = ie.y - (k2S.x * kap.y + k2S.y * kap.x);
    } else {
      const double rho = sqrt(double(d2));
      const double s = c0 / rho;
      double sn, cs;
      sincos(kh * rho, &sn, &cs);
      const double kr = s * cs, ki = -s * sn;  // K(d)
      z.x = -(kr * kap.x - ki * kap.y);
      z.y = -(kr * kap.y + ki * kap.x);
    }
    if (F32) F32[jb.f_off + e] = make_float2(float(z.x), float(z.y));
    if (F64) F64[jb.f_off + e] = z;
  }
}

void launch_entries(const EntryJob *jobs, int64_t njobs, const int32_t *cols, const short4 *xyz,
                    const double2 *inv_eps, const double2 *kappa, double kh, double2 k2S,
                    float2 *F32, double2 *F64, hipStream_t st) {
  for (int64_t j0 = 0; j0 < njobs; j0 += 1 << 30) {
    const int64_t nj = njobs - j0 < (1 << 30) ? njobs - j0 : (1 << 30);
    hipLaunchKernelGGL(k_entries, dim3(unsigned(nj)), dim3(256), 0, st, jobs + j0, cols, xyz,
                       inv_eps, kappa, kh, k2S, F32, F64);
  }
}

// ---------------------------------------------------------------------------
// Factor element loads: complex FP32, or a complex pair of 16-bit values packed as
// (re | im << 16) in BF16 or IEEE FP16.
struct FBF16 {
  uint32_t v;
};
struct FF16 {
  uint32_t v;
};
// Loads through global-address-space pointers (global_load rather than flat_load).
typedef float gfloat2v __attribute__((ext_vector_type(2)));
__device__ inline float2 ldg_f2(const float2 *p, int64_t idx) {
  const gfloat2v v = ((const __attribute__((address_space(1))) gfloat2v *)p)[idx];
  return make_float2(v.x, v.y);
}
// A uniform base plus a 32-bit byte offset per lane: the global_load's scalar-base form,
// with no 64-bit address arithmetic per lane.
__device__ inline float2 ldg_f2_sb(const float2 *base, uint32_t byte_off) {
  typedef const __attribute__((address_space(1))) char gchar;
  const gfloat2v v = *(const __attribute__((address_space(1))) gfloat2v *)((gchar *)base + byte_off);
  return make_float2(v.x, v.y);
}
__device__ inline uint32_t ldg_u32(const uint32_t *p, int64_t idx) {
  return ((const __attribute__((address_space(1))) uint32_t *)p)[idx];
}
__device__ inline float2 load_factor(const float2 *F, int64_t idx) { return ldg_f2(F, idx); }
__device__ inline float bf16_to_f(uint32_t h) { return __uint_as_float(h << 16); }
__device__ inline float2 load_factor(const FBF16 *F, int64_t idx) {
  const uint32_t w = ldg_u32(reinterpret_cast<const uint32_t *>(F), idx);
  return make_float2(bf16_to_f(w & 0xFFFFu), bf16_to_f(w >> 16));
}
__device__ inline float2 load_factor(const FF16 *F, int64_t idx) {
  const uint32_t w = ldg_u32(reinterpret_cast<const uint32_t *>(F), idx);
  return make_float2(__half2float(__ushort_as_half((unsigned short)(w & 0xFFFFu))),
                     __half2float(__ushort_as_half((unsigned short)(w >> 16))));
}

// Output row of local row r of a tile: the last row-map entry with start <= r.
__device__ __forceinline__ int64_t mapped_row(const RowMap *__restrict__ rm, int map0, int map1,
                                              int r) {
  int e = map0;
  for (int k = map0 + 1; k < map1; ++k)
    if (rm[k].start <= r) e = k;
  return int64_t(rm[e].out_row) + (r - rm[e].start);
}

// Small-R grouped GEMM: one wave per tile, 64 rows at a time.  Lanes split the rows
// and G = 64 / mp k-groups; factor columns are read coalesced, input values broadcast.
// Each lane keeps 8 factor loads in flight (columns k, k + G, ..., k + 7G) so the
// factor stream is not serialised on memory latency.
template <typename FT>
__global__ __launch_bounds__(256) void k_grouped_gemv(const Seg *__restrict__ segs,
                                                      const Pair *__restrict__ pairs,
                                                      const RowMap *__restrict__ rowmap,
                                                      const FT *__restrict__ F,
                                                      const float2 *__restrict__ X,
                                                      const float2 *__restrict__ T,
                                                      float2 *__restrict__ OUT, int R,
                                                      int beta, int64_t nseg) {
  constexpr int U = 8;
  const int64_t w = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (w >= nseg) return;
  const int lane = threadIdx.x & 63;
  const Seg sg = segs[w];
  for (int rb = 0; rb < sg.m; rb += 64) {
    const int m = sg.m - rb < 64 ? sg.m - rb : 64;
    const int mp = m <= 16 ? 16 : (m <= 32 ? 32 : 64);
    const int G = 64 / mp;
    const int i = lane % mp, g = lane / mp;
    const bool rok = i < m;
    for (int q0 = 0; q0 < R; q0 += 4) {
      const int nq = R - q0 < 4 ? R - q0 : 4;
      float ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
      for (int p = sg.p0; p < sg.p1; ++p) {
        const Pair pr = pairs[p];
        const float2 *in = (pr.in_buf ? T : X) + int64_t(pr.in_row) * R + q0;
        const FT *A = F + pr.f_off + rb;
        for (int k0 = g; k0 < pr.n; k0 += G * U) {
          float2 a[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int k = k0 + u * G;
            a[u] = (rok && k < pr.n) ? load_factor(A, int64_t(k) * pr.lda + i)
                                     : make_float2(0.f, 0.f);
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int k = k0 + u * G;
            if (k < pr.n) {
              const float2 *xk = in + int64_t(k) * R;
              const float2 av = make_float2(a[u].x * pr.scale, a[u].y * pr.scale);
#pragma unroll
              for (int qq = 0; qq < 4; ++qq) {
                if (qq < nq) {
                  const float2 x = xk[qq];
                  ar[qq] += av.x * x.x - av.y * x.y;
                  ai[qq] += av.x * x.y + av.y * x.x;
                }
              }
            }
          }
        }
      }
      for (int off = mp; off < 64; off <<= 1) {
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          ar[qq] += __shfl_xor(ar[qq], off);
          ai[qq] += __shfl_xor(ai[qq], off);
        }
      }
      if (g == 0 && rok) {
        float2 *o = OUT + mapped_row(rowmap, sg.map0, sg.map1, rb + i) * R + q0;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          if (qq < nq) {
            float2 v = make_float2(ar[qq], ai[qq]);
            if (beta) {
              const float2 u = o[qq];
              v.x += u.x;
              v.y += u.y;
            }
            o[qq] = v;
          }
        }
      }
    }
  }
}

// MFMA grouped GEMM with FP32 arithmetic (complex FP32 or FP16-stored factors).
// The complex product is one real GEMM: a factor row (ar_0, ai_0, ar_1, ai_1, ...)
// times Xt, where Xt row 2c holds (xr, xi) and row 2c+1 holds (-xi, xr) for every
// right-hand side, so output column pair (2q, 2q+1) is (Re y_q, Im y_q).
// v_mfma_f32_16x16x4f32: lane l holds A[l % 16][l / 16], B[l / 16][l % 16] and
// D[4 (l / 16) + v][l % 16].  Four MFMAs consume 8 complex columns: slot kk of MFMA t
// is real column 4 kk + t, i.e. complex column 2 kk + t / 2, part t % 2.
// One workgroup of kWaves waves owns one tile (<= kTileRows output rows).  Its output tiles
// (16 rows x 8 right-hand sides) are dealt to the waves as a cw x rw grid: wave w takes the
// column tiles congruent to w % cw and the row tiles congruent to w / cw, so every
// row count keeps all waves busy and a wave reuses its input fragments across its row
// tiles.  Factor columns and input rows are streamed in chunks of KC = 16 complex
// columns: each chunk is loaded once per workgroup, coalesced, into LDS; the next
// chunk is fetched into registers while the current one is multiplied.  The chunk
// loop is instantiated per (row tiles, column tiles) of a wave so that its inner
// loops have fixed trip counts; every instantiation runs the same barriers.
constexpr int kKC = 16;                 // complex K rows per chunk
constexpr int kXS = 68;                 // LDS stride of an input row (64 + 4 complex: conflict-free)
constexpr int kAS = kTileRows + 8;      // LDS stride of a factor column (conflict-free)
constexpr int kWaves = kTileRows / 16;  // waves per workgroup: one per row tile of a full tile
constexpr int kThreads = 64 * kWaves;
constexpr int kXL = kKC * 64 / kThreads;         // input elements per thread and chunk
constexpr int kAL = kKC * kTileRows / kThreads;  // factor elements per thread and chunk

// Where a chunk comes from: a pair's factor block and input rows, restricted to one
// right-hand-side slice [q0, q0 + rc) and the tile's m rows.  All fields are uniform.
struct ChunkSrc {
  int64_t x;  // element offset of input row 0, column q0, in X (xt = 0) or T (xt = 1)
  int64_t a;  // factor offset of the pair
  int xt, n, lda, rc, m;
  float scale;
};

__device__ __forceinline__ ChunkSrc chunk_src(const Pair &pr, int R, int q0, int rc, int m) {
  ChunkSrc c;
  c.x = int64_t(pr.in_row) * R + q0;
  c.xt = pr.in_buf;
  c.a = pr.f_off;
  c.n = pr.n;
  c.lda = pr.lda;
  c.rc = rc;
  c.m = m;
  c.scale = pr.scale;
  return c;
}


// Fetch chunk rows [kb, kb + kKC) of a source into registers.  Every lane loads from
// an in-bounds address (indices clamped to the block); bit i of msk says whether value i
// (inputs first, then factors) lies inside the block.  Masking and the factor scale are
// applied when the chunk is written to LDS, so the loads stay in flight until then.
template <typename FT>
__device__ __forceinline__ unsigned load_chunk(const ChunkSrc &c, int kb, const FT *__restrict__ F,
                                               const float2 *__restrict__ X,
                                               const float2 *__restrict__ T, int R,
                                               float2 (&xr)[kXL], float2 (&ar)[kAL]) {
  const int tid = threadIdx.x;
  const float2 *xb = (c.xt ? T : X) + c.x;
  const FT *ab = F + c.a;
  unsigned msk = 0;
#pragma unroll
  for (int i = 0; i < kXL; ++i) {
    const int e = tid + kThreads * i;
    const int hi = kb + (e >> 6), lo = e & 63;  // input row hi, column lo
    const unsigned off = unsigned(min(hi, c.n - 1)) * unsigned(R) + unsigned(min(lo, c.rc - 1));
    xr[i] = ldg_f2_sb(xb, off * 8u);
    msk |= unsigned(hi < c.n && lo < c.rc) << i;
  }
#pragma unroll
  for (int i = 0; i < kAL; ++i) {
    const int e = tid + kThreads * i;
    const int hi = kb + e / kTileRows, lo = e % kTileRows;  // factor column hi, row lo
    const unsigned off = unsigned(min(hi, c.n - 1)) * unsigned(c.lda) + unsigned(min(lo, c.m - 1));
    if constexpr (std::is_same<FT, float2>::value)
      ar[i] = ldg_f2_sb(ab, off * 8u);
    else
      ar[i] = load_factor(ab, off);
    msk |= unsigned(hi < c.n && lo < c.m) << (kXL + i);
  }
  return msk;
}

// Accumulators of one work item into its output rows.  The tile's row map (at most
// kMaxMapEntries entries, read with uniform loads; the array is padded past its end) is
// resolved per row in registers; accumulation into the output is a non-returning atomic
// add (each output element belongs to exactly one item, so it is a plain
// read-modify-write with nothing to wait on).
template <int NRI, int NCI, int RW>
__device__ __forceinline__ void store_item(const Seg &sg, const RowMap *__restrict__ rowmap,
                                           float2 *__restrict__ OUT, const int R, const int beta,
                                           const int q0, const int Rc, const int wr, const int wc,
                                           const floatx4 (&acc)[NRI > 0 ? NRI * NCI : 1]) {
  constexpr int CW = kWaves / RW;
  const int lane = threadIdx.x & 63;
  const int i16 = lane & 15, kk = lane >> 4;
  const int qo = i16 >> 1, op = i16 & 1;
  const int ne = sg.map1 - sg.map0;
  int mstart[kMaxMapEntries], mbase[kMaxMapEntries];
#pragma unroll
  for (int k = 0; k < kMaxMapEntries; ++k) {
    const RowMap e = rowmap[sg.map0 + k];
    mstart[k] = k < ne ? e.start : kTileRows;
    mbase[k] = e.out_row - e.start;
  }
#pragma unroll
  for (int ri = 0; ri < NRI; ++ri) {
    const int rt = wr + ri * RW;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = rt * 16 + 4 * kk + v;
      int base = mbase[0];
#pragma unroll
      for (int k = 1; k < kMaxMapEntries; ++k) base = mstart[k] <= row ? mbase[k] : base;
      if (row < sg.m) {
        const int64_t orow = int64_t(base) + row;
#pragma unroll
        for (int ci = 0; ci < NCI; ++ci) {
          const int q = q0 + (wc + ci * CW) * 8 + qo;
          if (q < q0 + Rc) {
            float *o = reinterpret_cast<float *>(OUT + orow * R + q) + op;
            if (beta)
              unsafeAtomicAdd(o, acc[ri * NCI + ci][v]);
            else
              *o = acc[ri * NCI + ci][v];
          }
        }
      }
    }
  }
}

// One work item: tile it / nsl with right-hand-side slice it % nsl of RQ (<= 64) columns.
// The wave owns NRI row tiles (wr, wr + RW, ...) and NCI column tiles (wc, wc + CW), CW =
// kWaves / RW; all LDS offsets are compile-time immediates from one lane base address.
// Factor columns and input rows stream through LDS in chunks of kKC; the next chunk
// (same pair, or the tile's next pair, whose descriptor is read one pair ahead) is
// fetched into registers while the current one is multiplied.
template <typename FT, int NRI, int NCI, int RW>
__device__ __forceinline__ void tile_item(const int it, const int nsl, const int RQ,
                                          const Seg *__restrict__ segs,
                                          const Pair *__restrict__ pairs,
                                          const RowMap *__restrict__ rowmap,
                                          const FT *__restrict__ F, const float2 *__restrict__ X,
                                          const float2 *__restrict__ T, float2 *__restrict__ OUT,
                                          const int R, const int beta, const int wr, const int wc,
                                          float2 *xs, float2 *as) {
  constexpr int CW = kWaves / RW;
  const int tid = threadIdx.x, lane = tid & 63;
  const int i16 = lane & 15;
  const int kk = lane >> 4;
  const int qo = i16 >> 1, op = i16 & 1;
  const float2 *xl = xs + 2 * kk * kXS + wc * 8 + qo;   // this lane's input fragment base
  const float2 *al = as + 2 * kk * kAS + wr * 16 + i16;  // this lane's factor fragment base
  const Seg sg = segs[it / nsl];
  const int q0 = (it % nsl) * RQ;
  const int Rc = min(R - q0, RQ);
  ChunkSrc cur = chunk_src(sg.first, R, q0, Rc, sg.m);
  float2 xr[kXL], ar[kAL];
  unsigned msk = load_chunk<FT>(cur, 0, F, X, T, R, xr, ar);
  float lscale = cur.scale;  // factor scale of the chunk held in xr / ar
  floatx4 acc[NRI > 0 ? NRI * NCI : 1];
#pragma unroll
  for (int j = 0; j < (NRI > 0 ? NRI * NCI : 1); ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
  int p = sg.p0, k0 = 0;
  Pair pr1;  // descriptor of the tile's following pair, fetched one pair ahead
  if (p + 1 < sg.p1) pr1 = pairs[p + 1];
  while (true) {
    __syncthreads();  // previous chunk fully consumed
#pragma unroll
    for (int i = 0; i < kXL; ++i) {
      const int e = tid + kThreads * i;
      const bool ok = (msk >> i) & 1u;
      xs[(e >> 6) * kXS + (e & 63)] = make_float2(ok ? xr[i].x : 0.f, ok ? xr[i].y : 0.f);
    }
#pragma unroll
    for (int i = 0; i < kAL; ++i) {
      const int e = tid + kThreads * i;
      const bool ok = (msk >> (kXL + i)) & 1u;
      as[(e / kTileRows) * kAS + e % kTileRows] =
          make_float2(ok ? ar[i].x * lscale : 0.f, ok ? ar[i].y * lscale : 0.f);
    }
    __syncthreads();
    // the second half of a chunk past the pair's last column holds only zeros
    const int nh = k0 + kKC / 2 < cur.n ? 2 : 1;
    // the next chunk: same pair, or the tile's next pair
    bool last = false;
    if (k0 + kKC < cur.n) {
      k0 += kKC;
    } else if (p + 1 < sg.p1) {
      ++p;
      k0 = 0;
      cur = chunk_src(pr1, R, q0, Rc, sg.m);
      if (p + 1 < sg.p1) pr1 = pairs[p + 1];
    } else {
      last = true;
    }
    if (!last) {
      msk = load_chunk<FT>(cur, k0, F, X, T, R, xr, ar);
      lscale = cur.scale;
    }
    if (NRI > 0) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h >= nh) break;
        // this lane's two complex K rows of the half chunk: 8 h + 2 kk and 8 h + 2 kk + 1
        float2 x0[NCI], x1[NCI];
#pragma unroll
        for (int ci = 0; ci < NCI; ++ci) {
          x0[ci] = xl[8 * h * kXS + ci * CW * 8];
          x1[ci] = xl[(8 * h + 1) * kXS + ci * CW * 8];
        }
        // row tiles in pairs when NCI = 1: every step interleaves at least two
        // accumulators, so no MFMA waits on the one just issued
        constexpr int JG = NCI == 1 && NRI > 1 ? 2 : 1;
#pragma unroll
        for (int j0 = 0; j0 < NRI; j0 += JG) {
          float2 a0[JG], a1[JG];
#pragma unroll
          for (int u = 0; u < JG; ++u) {
            const int j = j0 + u < NRI ? j0 + u : j0;
            a0[u] = al[8 * h * kAS + j * RW * 16];
            a1[u] = al[(8 * h + 1) * kAS + j * RW * 16];
          }
#pragma unroll
          for (int t = 0; t < 4; ++t) {
#pragma unroll
            for (int u = 0; u < JG; ++u) {
              if (j0 + u < NRI) {
                const float2 a = t < 2 ? a0[u] : a1[u];
                const float av = (t & 1) ? a.y : a.x;
#pragma unroll
                for (int ci = 0; ci < NCI; ++ci) {
                  const float2 x = t < 2 ? x0[ci] : x1[ci];
                  const float bv = (t & 1) ? (op ? x.x : -x.y) : (op ? x.y : x.x);
                  const int j = (j0 + u) * NCI + ci;
                  acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[j], 0, 0, 0);
                }
              }
            }
          }
        }
      }
    }
    if (last) break;
  }
  store_item<NRI, NCI, RW>(sg, rowmap, OUT, R, beta, q0, Rc, wr, wc, acc);
}

// Work index of this workgroup.  Blocks are dealt to the kNumXcd XCDs round-robin; here
// groups of kXcdGroup consecutive work indices are dealt instead (group j to XCD j mod
// kNumXcd, its members in consecutive slots of that XCD), so neighbouring tiles, which
// often read the same input rows, share an L2 while the load stays balanced.  gridDim.x
// is a multiple of kNumXcd * kXcdGroup.
constexpr int kNumXcd = 8, kXcdGroup = 8;
__device__ __forceinline__ int xcd_work_index() {
  const int x = int(blockIdx.x % kNumXcd), l = int(blockIdx.x / kNumXcd);
  return ((l / kXcdGroup) * kNumXcd + x) * kXcdGroup + l % kXcdGroup;
}

// Grouped launch: one workgroup per work item.  The tiles of a launch are sorted by their
// row-tile count nrt (classes 1..kWaves); class c holds the tiles [seg0[c], seg0[c + 1]),
// i.e. the work items [seg0[c] nsl, seg0[c + 1] nsl).  Within a class every wave has a
// fixed share of the tile's 16 x 8 output tiles, so one instantiation serves all of its
// items; a narrower last slice runs the full-slice instantiation (the extra column tiles
// read zeros and are not stored).
struct TileClasses {
  int seg0[kWaves + 1];
};

// The waves of a workgroup as a cw x rw grid for a tile of nrt row tiles: short tiles
// spread over column tiles, tall tiles over row tiles too; every wave then owns at most
// 4 row tiles x 2 column tiles.  sel = 2 nri + nci - 1 (0: no tiles) is wave-uniform.
struct WaveGrid {
  int rw, wr, wc, sel;
};
__device__ __forceinline__ WaveGrid wave_grid(int wave, int nrt, int R, int RQ) {
  const int nnt = ((R < RQ ? R : RQ) + 7) >> 3;  // column tiles of a full slice
  const int nntp = nnt >= 8 ? 8 : (nnt >= 4 ? 4 : (nnt >= 2 ? 2 : 1));
  const int cw = (kWaves == 8 && nrt > 2) || nntp > kWaves ? (nntp > 4 ? 4 : nntp) : nntp;
  WaveGrid g;
  g.rw = kWaves / cw;
  g.wc = wave % cw;
  g.wr = wave / cw;
  // row tiles wr, wr + rw, ... below nrt; column tiles wc, wc + cw below nnt (<= 2)
  const int nri = g.wr < nrt ? (nrt - g.wr + g.rw - 1) / g.rw : 0;
  const int nci = g.wc < nnt ? (g.wc + cw < nnt ? 2 : 1) : 0;
  g.sel = nci == 0 ? 0 : nri * 2 + (nci - 1);
  return g;
}

// One instantiation of HODBF_CLASS(row tiles, column tiles, wave rows) per wave shape.
#define HODBF_DISPATCH_CLASSES(g)                 \
  if ((g).rw == 1) {                              \
    switch ((g).sel) {                            \
      case 2: HODBF_CLASS(1, 1, 1); break;        \
      case 3: HODBF_CLASS(1, 2, 1); break;        \
      case 4: HODBF_CLASS(2, 1, 1); break;        \
      case 5: HODBF_CLASS(2, 2, 1); break;        \
      case 6: HODBF_CLASS(3, 1, 1); break;        \
      case 7: HODBF_CLASS(3, 2, 1); break;        \
      case 8: HODBF_CLASS(4, 1, 1); break;        \
      case 9: HODBF_CLASS(4, 2, 1); break;        \
      default: HODBF_CLASS(0, 1, 1); break;       \
    }                                             \
  } else if ((g).rw == 2) {                       \
    switch ((g).sel) {                            \
      case 2: HODBF_CLASS(1, 1, 2); break;        \
      case 3: HODBF_CLASS(1, 2, 2); break;        \
      case 4: HODBF_CLASS(2, 1, 2); break;        \
      case 5: HODBF_CLASS(2, 2, 2); break;        \
      default: HODBF_CLASS(0, 1, 2); break;       \
    }                                             \
  } else {                                        \
    if ((g).sel == 2) HODBF_CLASS(1, 1, 4);       \
    else HODBF_CLASS(0, 1, 4);                    \
  }

template <typename FT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_grouped_mfma_f32(
    const Seg *__restrict__ segs, const Pair *__restrict__ pairs, const RowMap *__restrict__ rowmap,
    const FT *__restrict__ F, const float2 *__restrict__ X, const float2 *__restrict__ T,
    float2 *__restrict__ OUT, int R, int beta, int RQ, int nsl, TileClasses tc) {
  __shared__ float2 xs[kKC * kXS];
  __shared__ float2 as[kKC * kAS];
  // neighbouring work on one XCD (see xcd_work_index); the padded grid's extra blocks exit
  const int it = xcd_work_index();
  if (it >= tc.seg0[kWaves] * nsl) return;
  int c = 0;
  while (c < kWaves - 1 && it >= tc.seg0[c + 1] * nsl) ++c;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const WaveGrid wg = wave_grid(wave, c + 1, R, RQ);
#define HODBF_CLASS(NR, NC, RWV)                                                             \
  tile_item<FT, NR, NC, RWV>(it, nsl, RQ, segs, pairs, rowmap, F, X, T, OUT, R, beta, wg.wr, \
                             wg.wc, xs, as)
  HODBF_DISPATCH_CLASSES(wg)
#undef HODBF_CLASS
}

// Split-BF16 arithmetic for complex FP32 factors and inputs.  Each FP32 value v is
// written as hi + lo with hi = bf16(v) and lo = bf16(v - hi), both rounded to nearest
// even, so |v - hi - lo| <= 2^-17 |v|; a product a x is taken as
// hi_a hi_x + hi_a lo_x + lo_a hi_x on v_mfma_f32_16x16x32_bf16 with FP32 accumulation:
// the dropped lo_a lo_x (at most 2^-16 |a x|) and the two split remainders (2^-17 each)
// keep it within 2^-15 |a| |x|.  One MFMA consumes a whole chunk of
// 16 complex columns (32 real K), against eight FP32 16x16x4 MFMAs of four times the
// cycles each: the same tiles, work items and chunk pipeline as tile_item, with the
// chunk split into hi / lo once, when it is written to LDS.
//
// Lane l = 16 kk + i16 supplies K slots 8 kk .. 8 kk + 7 of row / column i16 (the two
// operands use the same slot order, so the sum over K needs no particular hardware slot
// order).  Slots 2 v, 2 v + 1 are (Re, Im) of complex column 4 kk + v: for the factor
// that is the stored pair itself, for the input of output column 2 q it is (xr, -xi) and
// of column 2 q + 1 it is (xi, xr).  LDS holds the factor chunk row-major and the input
// chunk column-major in both forms, in the planes described below.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float floatx2v __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// LDS planes of the split-BF16 kernel (32-bit words): hi and lo parts apart, so that a
// fragment is one 16-byte read straight into the MFMA operand registers.  A plane holds
// 64 rows (factor) or 64 right-hand-side columns (input) of K = 0..15, packed
// (re | im << 16), in 16-byte units of four K values, K-group-major: the unit of row r
// and K group kk sits at unit kk * 64 + r.  gfx950 serves a 16-byte LDS read in four
// groups of 16 lanes, each holding every value of lane mod 16 once (lanes 0-3, 12-15,
// 20-23, 24-27; 4-7, 8-11, 16-19, 28-31; and the same pattern plus 32); a fragment's
// lane 16 kk + i16 reads row i16 of its row tile, so unit kk * 64 + r puts the 16 lanes of
// every group on distinct banks, and the staging stores of a wave (64 consecutive rows,
// one K group) are one contiguous kilobyte.  The second input form sits 8 units further
// modulo 16, so an input fragment's 8 columns x both forms cover distinct banks too.
constexpr int kS3Unit = 4;                 // words per unit
constexpr int kPlane = 4 * 64 * kS3Unit;   // words of one plane (4 K groups x 64 rows)
constexpr int kXF = 2 * kPlane + 32;       // words between the two input forms (hi + lo planes each)

// Chunk loads of the split-BF16 kernel: thread (lane l, wave g) fetches factor row l and
// input column l at K rows kb + 4 g .. kb + 4 g + 3, so that it can write its four values
// of each as one contiguous run (two 16-byte LDS stores).  Each load instruction still
// reads 64 consecutive rows of a factor column or 64 consecutive right-hand sides of an
// input row.  Indices are clamped into the block (the write to LDS zeroes what lies
// outside it).
__device__ __forceinline__ void load_chunk_t(const ChunkSrc &c, int kb, const float2 *__restrict__ F,
                                                 const float2 *__restrict__ X,
                                                 const float2 *__restrict__ T, int R,
                                                 float2 (&xr)[4], float2 (&ar)[4]) {
  const int l = threadIdx.x & 63;
  const int g = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const float2 *xb = (c.xt ? T : X) + c.x;
  const float2 *ab = F + c.a;
  const unsigned lq = unsigned(min(l, c.rc - 1)), lr = unsigned(min(l, c.m - 1));
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const unsigned kc = unsigned(min(kb + 4 * g + j, c.n - 1));
    xr[j] = ldg_f2_sb(xb, (kc * unsigned(R) + lq) * 8u);
    ar[j] = ldg_f2_sb(ab, (kc * unsigned(c.lda) + lr) * 8u);
  }
}

// (hi pair, lo pair) of the complex value (re, im), each packed re | im << 16
__device__ __forceinline__ uint2 split_bf16(float re, float im) {
  const floatx2v v = {re, im};
  const uint32_t hb = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2v));
  const float hre = __uint_as_float(hb << 16), him = __uint_as_float(hb & 0xFFFF0000u);
  const floatx2v r = {re - hre, im - him};
  const uint32_t lb = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf16x2v));
  return make_uint2(hb, lb);
}

template <int NRI, int NCI, int RW>
__device__ __forceinline__ void tile_item_s3(const int it, const int nsl, const int RQ,
                                             const Seg *__restrict__ segs,
                                             const Pair *__restrict__ pairs,
                                             const RowMap *__restrict__ rowmap,
                                             const float2 *__restrict__ F,
                                             const float2 *__restrict__ X,
                                             const float2 *__restrict__ T,
                                             float2 *__restrict__ OUT, const int R,
                                             const int beta, const int wr, const int wc,
                                             uint32_t *as, uint32_t *xs) {
  constexpr int CW = kWaves / RW;
  const int tid = threadIdx.x, lane = tid & 63;
  const int i16 = lane & 15;
  const int kk = lane >> 4;
  const int qo = i16 >> 1, op = i16 & 1;
  // this lane's fragment bases (hi planes; lo at + kPlane): factor row wr * 16 + i16, input
  // column wc * 8 + qo of form op, K group kk
  const uint32_t *al = as + (kk * 64 + wr * 16 + i16) * kS3Unit;
  const uint32_t *xl = xs + op * kXF + (kk * 64 + wc * 8 + qo) * kS3Unit;
  const Seg sg = segs[it / nsl];
  const int q0 = (it % nsl) * RQ;
  const int Rc = min(R - q0, RQ);
  floatx4 acc[NRI > 0 ? NRI * NCI : 1];
#pragma unroll
  for (int j = 0; j < (NRI > 0 ? NRI * NCI : 1); ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
  // The load cursor (pair p, column k0, source cur) runs one chunk ahead of the chunk
  // being multiplied: its loads are in flight during the multiply.  (Two chunks ahead in
  // two register sets measured no faster and costs the fifth wave per SIMD.)
  ChunkSrc cur = chunk_src(sg.first, R, q0, Rc, sg.m);
  int p = sg.p0, k0 = 0;
  bool done = false;
  Pair pr1;  // descriptor of pair p + 1
  if (p + 1 < sg.p1) pr1 = pairs[p + 1];
  auto advance = [&]() {
    if (k0 + kKC < cur.n) {
      k0 += kKC;
    } else if (p + 1 < sg.p1) {
      ++p;
      k0 = 0;
      cur = chunk_src(pr1, R, q0, Rc, sg.m);
      if (p + 1 < sg.p1) pr1 = pairs[p + 1];
    } else {
      done = true;
    }
  };
  // thread (l, g) writes K = 4 g .. 4 g + 3 of factor row l and of input column l: one
  // 16-byte store per plane
  // values outside the block (K row kb + 4 g + j past the pair's columns: a wave-uniform
  // test; lane l past the slice's columns or the tile's rows) are written as zeros
  auto write_chunk = [&](const float2 (&xr)[4], const float2 (&ar)[4], const ChunkSrc &c,
                         int kb) {
    const int l = tid & 63;
    const int g = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool lx = l < c.rc, la = l < c.m;
    uint2 h[4], a[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool kv = kb + 4 * g + j < c.n;
      const bool okx = kv && lx, oka = kv && la;
      h[j] = split_bf16(okx ? xr[j].x : 0.f, okx ? xr[j].y : 0.f);
      a[j] = split_bf16(oka ? ar[j].x * c.scale : 0.f, oka ? ar[j].y * c.scale : 0.f);
    }
    const int o = (g * 64 + l) * kS3Unit;
    constexpr uint32_t sg = 0x80000000u;
    auto rot = [](uint32_t v) { return __builtin_amdgcn_alignbit(v, v, 16); };
    *reinterpret_cast<u32x4 *>(as + o) = u32x4{a[0].x, a[1].x, a[2].x, a[3].x};
    *reinterpret_cast<u32x4 *>(as + kPlane + o) = u32x4{a[0].y, a[1].y, a[2].y, a[3].y};
    // form 0: (xr, -xi); form 1: (xi, xr)
    *reinterpret_cast<u32x4 *>(xs + o) = u32x4{h[0].x ^ sg, h[1].x ^ sg, h[2].x ^ sg, h[3].x ^ sg};
    *reinterpret_cast<u32x4 *>(xs + kPlane + o) =
        u32x4{h[0].y ^ sg, h[1].y ^ sg, h[2].y ^ sg, h[3].y ^ sg};
    *reinterpret_cast<u32x4 *>(xs + kXF + o) = u32x4{rot(h[0].x), rot(h[1].x), rot(h[2].x), rot(h[3].x)};
    *reinterpret_cast<u32x4 *>(xs + kXF + kPlane + o) =
        u32x4{rot(h[0].y), rot(h[1].y), rot(h[2].y), rot(h[3].y)};
  };
  auto multiply = [&]() {
    if (NRI > 0) {
      bf16x8 xh[NCI], xo[NCI];
#pragma unroll
      for (int ci = 0; ci < NCI; ++ci) {
        const uint32_t *b = xl + ci * CW * 8 * kS3Unit;
        xh[ci] = *reinterpret_cast<const bf16x8 *>(b);
        xo[ci] = *reinterpret_cast<const bf16x8 *>(b + kPlane);
      }
      // one row tile at a time (its fragments are used by NCI column tiles); within it the
      // three products run term-major, so consecutive MFMAs alternate accumulators
#pragma unroll
      for (int ri = 0; ri < NRI; ++ri) {
        const uint32_t *a = al + ri * RW * 16 * kS3Unit;
        const bf16x8 ah = *reinterpret_cast<const bf16x8 *>(a);
        const bf16x8 ao = *reinterpret_cast<const bf16x8 *>(a + kPlane);
#pragma unroll
        for (int ci = 0; ci < NCI; ++ci)
          acc[ri * NCI + ci] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, xh[ci], acc[ri * NCI + ci], 0, 0, 0);
#pragma unroll
        for (int ci = 0; ci < NCI; ++ci)
          acc[ri * NCI + ci] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, xo[ci], acc[ri * NCI + ci], 0, 0, 0);
#pragma unroll
        for (int ci = 0; ci < NCI; ++ci)
          acc[ri * NCI + ci] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(ao, xh[ci], acc[ri * NCI + ci], 0, 0, 0);
      }
    }
  };
  // the registers' chunk keeps its uniform source and first column; the lane masks are
  // recomputed from them when it is written to LDS
  float2 xr[4], ar[4];
  ChunkSrc cc = cur;
  int kbc = k0;
  load_chunk_t(cur, k0, F, X, T, R, xr, ar);
  while (true) {
    __syncthreads();
    write_chunk(xr, ar, cc, kbc);
    __syncthreads();
    advance();
    const bool more = !done;
    cc = cur;
    kbc = k0;
    if (more) load_chunk_t(cur, k0, F, X, T, R, xr, ar);
    multiply();
    if (!more) break;
  }
  store_item<NRI, NCI, RW>(sg, rowmap, OUT, R, beta, q0, Rc, wr, wc, acc);
}

// Six waves per SIMD (80 VGPRs, no spills; six workgroups' 24.7 KB of LDS fit a CU's
// 160 KB): 1-2% faster than five at 1-64 right-hand sides, and five faster than four at
// 1-16.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_grouped_mfma_s3(
    const Seg *__restrict__ segs, const Pair *__restrict__ pairs, const RowMap *__restrict__ rowmap,
    const float2 *__restrict__ F, const float2 *__restrict__ X, const float2 *__restrict__ T,
    float2 *__restrict__ OUT, int R, int beta, int RQ, int nsl, TileClasses tc) {
  static_assert(kTileRows == 64, "one plane row per tile row");
  __shared__ __attribute__((aligned(16))) uint32_t as[2 * kPlane];
  __shared__ __attribute__((aligned(16))) uint32_t xs[kXF + 2 * kPlane];
  const int it = xcd_work_index();
  if (it >= tc.seg0[kWaves] * nsl) return;
  int c = 0;
  while (c < kWaves - 1 && it >= tc.seg0[c + 1] * nsl) ++c;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const WaveGrid wg = wave_grid(wave, c + 1, R, RQ);
#define HODBF_CLASS(NR, NC, RWV)                                                              \
  tile_item_s3<NR, NC, RWV>(it, nsl, RQ, segs, pairs, rowmap, F, X, T, OUT, R, beta, wg.wr, wg.wc, \
                            as, xs)
  HODBF_DISPATCH_CLASSES(wg)
#undef HODBF_CLASS
}

// MFMA grouped GEMM, complex BF16 factors (v_mfma_f32_16x16x16bf16_1k): one MFMA
// consumes 8 complex columns; lane slot kk holds real columns 4 kk .. 4 kk + 3, i.e.
// (Re, Im) of complex columns 2 kk and 2 kk + 1.  Inputs are rounded to BF16 with
// round-to-nearest-even; accumulation is FP32.  The tile is processed 64 rows at a time.
__device__ inline short f_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return short(u >> 16);
}

__global__ __launch_bounds__(256) void k_grouped_mfma_bf16(const Seg *__restrict__ segs,
                                                           const Pair *__restrict__ pairs,
                                                           const RowMap *__restrict__ rowmap,
                                                           const uint32_t *__restrict__ F,
                                                           const float2 *__restrict__ X,
                                                           const float2 *__restrict__ T,
                                                           float2 *__restrict__ OUT, int R,
                                                           int beta) {
  const Seg sg = segs[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kk = lane >> 4;
  const int jc = lane & 15;
  const int qo = jc >> 1, op = jc & 1;
  for (int rb = 0; rb < sg.m; rb += 64) {
    const int m = sg.m - rb < 64 ? sg.m - rb : 64;
    const int nrt = (m + 15) >> 4;
    const int nrtp = nrt == 3 ? 4 : nrt;
    const int wpr = 4 / nrtp;
    const int rt = wave / wpr;
    if (rt >= nrt) continue;
    const int sub = wave % wpr;
    const int ia = rt * 16 + (lane & 15);
    for (int q0 = 0; q0 < R; q0 += 64) {
      const int Rc = R - q0 < 64 ? R - q0 : 64;
      const int nnt = (Rc + 7) >> 3;
      floatx4 acc[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
      for (int p = sg.p0; p < sg.p1; ++p) {
        const Pair pr = pairs[p];
        const uint32_t *A = F + pr.f_off + rb;
        const float2 *in = (pr.in_buf ? T : X) + int64_t(pr.in_row) * R;
        const int n = pr.n;
        const float sc = pr.scale;  // applied to the inputs: the BF16 MFMA has no per-pair scale
        for (int c0 = 0; c0 < n; c0 += 8) {
          const int c = c0 + 2 * kk;
          const bool rok = ia < m;
          const uint32_t w0 = (rok && c < n) ? A[int64_t(c) * pr.lda + ia] : 0u;
          const uint32_t w1 = (rok && c + 1 < n) ? A[int64_t(c + 1) * pr.lda + ia] : 0u;
          shortx4 av;
          av[0] = short(w0 & 0xFFFFu);
          av[1] = short(w0 >> 16);
          av[2] = short(w1 & 0xFFFFu);
          av[3] = short(w1 >> 16);
          const float2 z2 = make_float2(0.f, 0.f);
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int nt = sub + j * wpr;
            if (nt < nnt) {
              const int q = q0 + nt * 8 + qo;
              const bool qok = q < R;
              float2 x0 = (qok && c < n) ? in[int64_t(c) * R + q] : z2;
              float2 x1 = (qok && c + 1 < n) ? in[int64_t(c + 1) * R + q] : z2;
              x0.x *= sc;
              x0.y *= sc;
              x1.x *= sc;
              x1.y *= sc;
              shortx4 bv;
              bv[0] = f_to_bf16(op ? x0.y : x0.x);
              bv[1] = f_to_bf16(op ? x0.x : -x0.y);
              bv[2] = f_to_bf16(op ? x1.y : x1.x);
              bv[3] = f_to_bf16(op ? x1.x : -x1.y);
              acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[j], 0, 0, 0);
            }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int nt = sub + j * wpr;
        if (nt < nnt) {
          const int q = q0 + nt * 8 + qo;
          if (q < R) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = rt * 16 + 4 * kk + v;
              if (row < m) {
                const int64_t orow = mapped_row(rowmap, sg.map0, sg.map1, rb + row);
                float *o = reinterpret_cast<float *>(OUT + orow * R + q) + op;
                *o = beta ? *o + acc[j][v] : acc[j][v];
              }
            }
          }
        }
      }
    }
  }
}

void launch_grouped(const Seg *segs, const Pair *pairs, const RowMap *rowmap, int64_t s0,
                    int64_t ns, const int64_t *cls, const void *F, int ftype, const float2 *X,
                    const float2 *T, float2 *OUT, int R, int beta, hipStream_t st) {
  if (ns <= 0 || R <= 0) return;
  const Seg *sp = segs + s0;
  // FP32 and FP16-stored factors take the MFMA kernel at every R (at R < 8 its extra
  // column tiles read clamped inputs and are not stored: MFMA work is wasted, but a
  // product with few columns is bound by streaming the factors, which that kernel does
  // best); BF16 factors below 4 columns use the vector kernel.
  if (R < 4 && ftype == FT_BF16) {
    const int64_t nb = (ns + 3) / 4;
    hipLaunchKernelGGL(k_grouped_gemv<FBF16>, dim3(unsigned(nb)), dim3(256), 0, st, sp, pairs,
                       rowmap, static_cast<const FBF16 *>(F), X, T, OUT, R, beta, ns);
    return;
  }
  if (ftype == FT_BF16) {
    hipLaunchKernelGGL(k_grouped_mfma_bf16, dim3(unsigned(ns)), dim3(256), 0, st, sp, pairs,
                       rowmap, static_cast<const uint32_t *>(F), X, T, OUT, R, beta);
    return;
  }
  // right-hand-side slice per work item: 64, or narrower when a launch has too few
  // tiles to give every SIMD several waves
  static const int64_t min_wg = [] {
    const char *e = std::getenv("HODBF_MIN_WORKGROUPS");  // tuning knob, default 512
    return e ? std::atoll(e) : int64_t(512);
  }();
  int RQ = 64;
  while (RQ > 16 && ns * ((R + RQ - 1) / RQ) < min_wg) RQ >>= 1;
  if (RQ > R) RQ = R;
  const int nsl = (R + RQ - 1) / RQ;
  TileClasses tc{};
  for (int c = 0; c <= kRowClasses; ++c) tc.seg0[c] = int(cls[c]);
  const int64_t items = ns * nsl;  // one workgroup per work item
  constexpr int64_t gq = kNumXcd * kXcdGroup;
  const dim3 grid{unsigned((items + gq - 1) / gq * gq)};
  if (ftype == FT_C64)
    hipLaunchKernelGGL(k_grouped_mfma_f32<float2>, grid, dim3(kThreads), 0, st, sp, pairs, rowmap,
                       static_cast<const float2 *>(F), X, T, OUT, R, beta, RQ, nsl, tc);
  else if (ftype == FT_C64_S3)
    hipLaunchKernelGGL(k_grouped_mfma_s3, grid, dim3(kThreads), 0, st, sp, pairs, rowmap,
                       static_cast<const float2 *>(F), X, T, OUT, R, beta, RQ, nsl, tc);
  else
    hipLaunchKernelGGL(k_grouped_mfma_f32<FF16>, grid, dim3(kThreads), 0, st, sp, pairs, rowmap,
                       static_cast<const FF16 *>(F), X, T, OUT, R, beta, RQ, nsl, tc);
}

// ---------------------------------------------------------------------------
// Permutation between the user's column-major order and the internal tree-order,
// RHS-interleaved layout, staged through LDS so both sides are read / written in runs.
template <typename S, typename D>
__device__ inline D cvt(S v);
template <>
__device__ inline float2 cvt<float2, float2>(float2 v) { return v; }
template <>
__device__ inline double2 cvt<double2, double2>(double2 v) { return v; }
template <>
__device__ inline float2 cvt<double2, float2>(double2 v) {
  return make_float2(float(v.x), float(v.y));
}
template <>
__device__ inline double2 cvt<float2, double2>(float2 v) {
  return make_double2(double(v.x), double(v.y));
}

// A workgroup takes 64 consecutive user indices u and 32 right-hand sides.  The user
// side moves one column's 64 elements as one contiguous run per wave; the tree side
// moves one element's 32 right-hand sides as one contiguous run at tree position
// tpos[u].
template <typename S, typename D>
__global__ __launch_bounds__(256) void k_gather(const S *__restrict__ src, int64_t ld,
                                                D *__restrict__ dst,
                                                const int32_t *__restrict__ tpos, int64_t n,
                                                int R) {
  __shared__ D tile[64][33];
  const int64_t u0 = int64_t(blockIdx.x) * 64;
  const int q0 = blockIdx.y * 32;
  for (int e = threadIdx.x; e < 64 * 32; e += 256) {
    const int ul = e & 63, ql = e >> 6;
    const int64_t u = u0 + ul;
    const int q = q0 + ql;
    if (u < n && q < R) tile[ul][ql] = cvt<S, D>(src[u + int64_t(q) * ld]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 32; e += 256) {
    const int ql = e & 31, ul = e >> 5;
    const int64_t u = u0 + ul;
    const int q = q0 + ql;
    if (u < n && q < R) dst[int64_t(tpos[u]) * R + q] = tile[ul][ql];
  }
}

// The reverse direction keeps tree rows as the staged unit: a workgroup takes 64
// consecutive tree positions and 32 right-hand sides, reads each position's 32 values as
// one run and writes user index perm[i] of each column (measured faster than the
// gather's arrangement for this direction).
template <typename S, typename D>
__global__ __launch_bounds__(256) void k_scatter(const S *__restrict__ src, D *__restrict__ dst,
                                                 int64_t ld, const int32_t *__restrict__ perm,
                                                 int64_t n, int R) {
  __shared__ D tile[64][33];
  const int64_t i0 = int64_t(blockIdx.x) * 64;
  const int q0 = blockIdx.y * 32;
  for (int e = threadIdx.x; e < 64 * 32; e += 256) {
    const int ql = e & 31, il = e >> 5;
    const int64_t i = i0 + il;
    const int q = q0 + ql;
    if (i < n && q < R) tile[il][ql] = cvt<S, D>(src[i * R + q]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 32; e += 256) {
    const int il = e & 63, ql = e >> 6;
    const int64_t i = i0 + il;
    const int q = q0 + ql;
    if (i < n && q < R) dst[int64_t(perm[i]) + int64_t(q) * ld] = tile[il][ql];
  }
}

void launch_gather(const void *src, bool src_c128, int64_t ld, void *dst, bool dst_c128,
                   const int32_t *tpos, int64_t n, int R, hipStream_t st) {
  if (n <= 0 || R <= 0) return;
  dim3 grid(unsigned((n + 63) / 64), unsigned((R + 31) / 32));
  if (src_c128 && dst_c128)
    hipLaunchKernelGGL((k_gather<double2, double2>), grid, dim3(256), 0, st,
                       (const double2 *)src, ld, (double2 *)dst, tpos, n, R);
  else if (src_c128)
    hipLaunchKernelGGL((k_gather<double2, float2>), grid, dim3(256), 0, st,
                       (const double2 *)src, ld, (float2 *)dst, tpos, n, R);
  else if (dst_c128)
    hipLaunchKernelGGL((k_gather<float2, double2>), grid, dim3(256), 0, st,
                       (const float2 *)src, ld, (double2 *)dst, tpos, n, R);
  else
    hipLaunchKernelGGL((k_gather<float2, float2>), grid, dim3(256), 0, st, (const float2 *)src,
                       ld, (float2 *)dst, tpos, n, R);
}

void launch_scatter(const void *src, bool src_c128, void *dst, bool dst_c128, int64_t ld,
                    const int32_t *perm, int64_t n, int R, hipStream_t st) {
  if (n <= 0 || R <= 0) return;
  dim3 grid(unsigned((n + 63) / 64), unsigned((R + 31) / 32));
  if (src_c128 && dst_c128)
    hipLaunchKernelGGL((k_scatter<double2, double2>), grid, dim3(256), 0, st,
                       (const double2 *)src, (double2 *)dst, ld, perm, n, R);
  else if (src_c128)
    hipLaunchKernelGGL((k_scatter<double2, float2>), grid, dim3(256), 0, st,
                       (const double2 *)src, (float2 *)dst, ld, perm, n, R);
  else if (dst_c128)
    hipLaunchKernelGGL((k_scatter<float2, double2>), grid, dim3(256), 0, st,
                       (const float2 *)src, (double2 *)dst, ld, perm, n, R);
  else
    hipLaunchKernelGGL((k_scatter<float2, float2>), grid, dim3(256), 0, st, (const float2 *)src,
                       (float2 *)dst, ld, perm, n, R);
}

// ---------------------------------------------------------------------------
// Plane-wave excitation (Section IV): b(i, q) = exp(-j k0 dhat_q . (r_i - r_c)).
__global__ __launch_bounds__(256) void k_plane_wave(const double *__restrict__ dirs, int R,
                                                    int nx, int ny, int nz, double h, double k0,
                                                    double2 *__restrict__ b, int64_t ldb) {
  const int64_t n = int64_t(nx) * ny * nz;
  const int q = blockIdx.y;
  const double dx = dirs[3 * q], dy = dirs[3 * q + 1], dz = dirs[3 * q + 2];
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int ix = int(i % nx), iy = int((i / nx) % ny), iz = int(i / (int64_t(nx) * ny));
    const double rx = h * (ix + 0.5 - 0.5 * nx), ry = h * (iy + 0.5 - 0.5 * ny),
                 rz = h * (iz + 0.5 - 0.5 * nz);
    double s, c;
    sincos(-k0 * (dx * rx + dy * ry + dz * rz), &s, &c);
    b[i + int64_t(q) * ldb] = make_double2(c, s);
  }
}

void launch_plane_wave(const double *dirs_dev, int R, int nx, int ny, int nz, double h,
                       double k0, double2 *b, int64_t ldb, hipStream_t st) {
  const int64_t n = int64_t(nx) * ny * nz;
  if (n <= 0 || R <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_plane_wave, dim3(unsigned(blocks), unsigned(R)), dim3(256), 0, st,
                     dirs_dev, R, nx, ny, nz, h, k0, b, ldb);
}

}  // namespace hodbf
