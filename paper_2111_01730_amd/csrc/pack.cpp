// Packing of butterfly factors into device programs: stage-by-stage grouped launches
// (all butterflies of a set advance one level per launch) and a final per-leaf reduce
// that applies the outer factors B^L (and the dense leaf blocks for Z_con).
//
// Blocks that read the same input rows are stacked into one matrix so the input is
// streamed once: at the first stage every V^0 block whose column leaf is nu (one per
// butterfly level), at later stages the two transfer blocks W_{tau1,nu} and
// W_{tau2,nu} of sibling row clusters, whose input is the same [t(p,nu1); t(p,nu2)].
// Each stacked matrix is cut into balanced tiles of at most kTileRows rows whose row
// maps scatter the rows back to each block's own output range.
#include <algorithm>
#include <functional>
#include <map>
#include <set>
#include <tuple>

#include "pack_sink.h"

namespace hodbf {

namespace {

struct Member {
  const Mat *f;
  int64_t out_row;
  int64_t kind, md[4], s, a, b;
};

// Stack the members (same n) into one column-major matrix and emit its tiles.
void emit_group(PackSink &pk, const std::vector<Member> &mem, int32_t in_buf, int64_t in_row,
                int64_t n) {
  int64_t mt = 0;
  for (auto &m : mem) mt += m.f->m;
  if (mt == 0 || n == 0) return;
  Mat S;
  S.m = int(mt);
  S.n = int(n);
  S.v.resize(size_t(mt) * size_t(n));
  std::vector<int64_t> roff;
  int64_t r = 0;
  for (auto &m : mem) {
    roff.push_back(r);
    for (int64_t k = 0; k < n; ++k)
      for (int64_t i = 0; i < m.f->m; ++i)
        S.v[size_t(k * mt + r + i)] = m.f->v[size_t(k * m.f->m + i)];
    r += m.f->m;
  }
  float scale = 1.0f;
  const int64_t f_off = pk.put_host(S, &scale);
  for (size_t j = 0; j < mem.size(); ++j) {
    const Member &m = mem[j];
    if (m.f->m == 0) continue;
    pk.table->push_back({m.kind, m.md[0], m.md[1], m.md[2], m.md[3], m.s, m.a, m.b, m.f->m, n,
                         f_off + roff[j], mt});
    if (pk.scales) pk.scales->push_back(scale);
  }
  // balanced tiles whose row counts are multiples of the 16-row MFMA tile (but the last),
  // cut early where a tile would span more than kMaxMapEntries blocks
  const int64_t ntile = (mt + kTileRows - 1) / kTileRows;
  const int64_t per = ((mt + 15) / 16 + ntile - 1) / ntile * 16;
  for (int64_t r0 = 0, r1 = 0; r0 < mt; r0 = r1) {
    r1 = std::min(mt, r0 + per);
    int spanned = 0;
    for (size_t j = 0; j < mem.size(); ++j) {
      const int64_t a0 = roff[j], a1 = roff[j] + mem[j].f->m;
      if (a1 <= r0 || a0 >= r1) continue;
      if (++spanned > kMaxMapEntries) {
        r1 = a0;
        break;
      }
    }
    Seg sg{};
    sg.m = int32_t(r1 - r0);
    sg.p0 = int32_t(pk.pairs.size());
    Pair p{};
    p.f_off = f_off + r0;
    p.in_row = int32_t(in_row);
    p.n = int32_t(n);
    p.lda = int32_t(mt);
    p.in_buf = in_buf;
    p.scale = scale;
    pk.pairs.push_back(p);
    sg.p1 = int32_t(pk.pairs.size());
    sg.map0 = int32_t(pk.rowmap.size());
    for (size_t j = 0; j < mem.size(); ++j) {
      const int64_t a0 = roff[j], a1 = roff[j] + mem[j].f->m;
      if (a1 <= r0 || a0 >= r1) continue;
      const int64_t st = std::max(a0, r0);
      pk.rowmap.push_back({int32_t(st - r0), int32_t(mem[j].out_row + (st - a0))});
    }
    sg.map1 = int32_t(pk.rowmap.size());
    pk.segs.push_back(sg);
  }
}

}  // namespace

// Re-emit every launch's tiles; in a launch with fewer than `below` tiles, a tile taller
// than `rows` is cut into tiles of at most `rows` rows (each keeps all of its pairs,
// offset to its rows, and the matching part of its row map).  Row tiles re-read only
// the (small) input rows, where right-hand-side slices would re-read the factors.
void retile(PackSink &pk, int64_t below, int rows) {
  std::vector<Seg> segs;
  std::vector<Pair> pairs;
  std::vector<RowMap> maps;
  segs.reserve(pk.segs.size());
  pairs.reserve(pk.pairs.size());
  maps.reserve(pk.rowmap.size());
  for (Launch &ln : pk.launches) {
    const int32_t lim = ln.ns < below ? rows : kTileRows;
    const int64_t s0 = int64_t(segs.size());
    for (int64_t si = ln.s0; si < ln.s0 + ln.ns; ++si) {
      const Seg &s = pk.segs[size_t(si)];
      for (int32_t r0 = 0; r0 < s.m || (s.m == 0 && r0 == 0); r0 += lim) {
        const int32_t r1 = std::min(s.m, r0 + lim);
        Seg t{};
        t.m = r1 - r0;
        t.p0 = int32_t(pairs.size());
        for (int32_t p = s.p0; p < s.p1; ++p) {
          Pair q = pk.pairs[size_t(p)];
          q.f_off += r0;  // column-major blocks: the tile's rows start r0 further
          pairs.push_back(q);
        }
        t.p1 = int32_t(pairs.size());
        t.map0 = int32_t(maps.size());
        for (int32_t e = s.map0; e < s.map1; ++e) {
          const RowMap &me = pk.rowmap[size_t(e)];
          const int32_t end = e + 1 < s.map1 ? pk.rowmap[size_t(e + 1)].start : s.m;
          if (end <= r0 || me.start >= std::max(r1, r0 + 1)) continue;
          const int32_t st = std::max(me.start, r0);
          maps.push_back({st - r0, me.out_row + (st - me.start)});
        }
        t.map1 = int32_t(maps.size());
        segs.push_back(t);
        if (s.m == 0) break;
      }
    }
    ln.s0 = s0;
    ln.ns = int64_t(segs.size()) - s0;
  }
  pk.segs.swap(segs);
  pk.pairs.swap(pairs);
  pk.rowmap.swap(maps);
}

// Pack one set of butterflies whose row and column trees end at the leaves of T_H.
// meta(bf) gives (l, i, ca, cb) for the block table.
void pack_group(PackSink &pk, const Tree &t, const std::vector<const Butterfly *> &bfs,
                bool forward, int final_beta,
                const std::function<void(const Butterfly &, int64_t *)> &meta) {
  // the leaf level of every butterfly of the set: the tree's leaves, or a coarser level
  // for the butterflies of the inverse's recursion (their leaf clusters may exceed a tile)
  int LH = t.depth;
  if (!bfs.empty()) LH = bfs[0]->hod_level + bfs[0]->L;
  for (auto *bf : bfs)
    if (bf->hod_level + bf->L != LH) fail(HODBF_E_ARG, "butterflies of one program must share a leaf level");
  if (forward && LH != t.depth) fail(HODBF_E_ARG, "dense leaf blocks need the tree's leaves");
  int Lmax = -1;
  for (auto *bf : bfs) Lmax = std::max(Lmax, bf->L);
  // off[k][s][idx]: first workspace row of output (a, b) at stage s of butterfly k
  std::vector<std::vector<std::vector<int64_t>>> off(bfs.size());
  for (size_t k = 0; k < bfs.size(); ++k) off[k].resize(bfs[k]->L + 1);
  const int64_t nleaf = int64_t(1) << LH;
  for (int s = 0; s <= Lmax; ++s) {
    const int64_t seg0 = int64_t(pk.segs.size());
    // workspace rows of this stage: butterfly-major, then a-major, b-minor
    for (size_t k = 0; k < bfs.size(); ++k) {
      const Butterfly &bf = *bfs[k];
      if (bf.L < s) continue;
      const int64_t na = int64_t(1) << s, nb = int64_t(1) << (bf.L - s);
      off[k][s].resize(size_t(na * nb));
      for (int64_t e = 0; e < na * nb; ++e) {
        const Mat &f = s == 0 ? bf.V0[size_t(e)] : bf.W[s][size_t(e)];
        off[k][s][size_t(e)] = pk.t_rows;
        pk.t_rows += f.m;
      }
    }
    if (s == 0) {
      // group V^0 blocks by their input leaf
      std::vector<std::vector<Member>> byleaf(static_cast<size_t>(nleaf));
      for (size_t k = 0; k < bfs.size(); ++k) {
        const Butterfly &bf = *bfs[k];
        int64_t md[4];
        meta(bf, md);
        for (int64_t b = 0; b < (int64_t(1) << bf.L); ++b) {
          const Mat &f = bf.V0[size_t(b)];
          if (f.m == 0 || f.n == 0) continue;
          const int64_t nu = (bf.si << bf.L) + b;
          byleaf[size_t(nu)].push_back(
              {&f, off[k][0][size_t(b)], 1, {md[0], md[1], md[2], md[3]}, 0, 0, b});
        }
      }
      for (int64_t nu = 0; nu < nleaf; ++nu)
        if (!byleaf[size_t(nu)].empty())
          emit_group(pk, byleaf[size_t(nu)], 0, t.node_lo(LH, nu),
                     t.node_hi(LH, nu) - t.node_lo(LH, nu));
    } else {
      // group the two sibling transfer blocks that read the same input segment
      for (size_t k = 0; k < bfs.size(); ++k) {
        const Butterfly &bf = *bfs[k];
        if (bf.L < s) continue;
        int64_t md[4];
        meta(bf, md);
        const int64_t nb = int64_t(1) << (bf.L - s);
        for (int64_t ap = 0; ap < (int64_t(1) << (s - 1)); ++ap)
          for (int64_t b = 0; b < nb; ++b) {
            std::vector<Member> mem;
            int64_t n = 0;
            for (int c = 0; c < 2; ++c) {
              const int64_t a = 2 * ap + c;
              const Mat &f = bf.W[s][size_t(a * nb + b)];
              n = f.n;
              if (f.m == 0 || f.n == 0) continue;
              mem.push_back(
                  {&f, off[k][s][size_t(a * nb + b)], 2, {md[0], md[1], md[2], md[3]}, s, a, b});
            }
            if (!mem.empty())
              emit_group(pk, mem, 1, off[k][s - 1][size_t(ap * 2 * nb + 2 * b)], n);
          }
      }
    }
    const int64_t ns = int64_t(pk.segs.size()) - seg0;
    if (ns > 0) pk.launches.push_back({seg0, ns, 0, 0});
  }
  // final reduce: every leaf g gets its dense block (forward) and one outer block B_a
  // from each butterfly whose row tree holds g
  std::vector<std::vector<std::pair<int, int64_t>>> cover(static_cast<size_t>(nleaf));
  for (size_t k = 0; k < bfs.size(); ++k) {
    const Butterfly &bf = *bfs[k];
    for (int64_t a = 0; a < (int64_t(1) << bf.L); ++a)
      cover[size_t((bf.oi << bf.L) + a)].push_back({int(k), a});
  }
  const int64_t seg0 = int64_t(pk.segs.size());
  for (int64_t g = 0; g < nleaf; ++g) {
    const int32_t lo = t.node_lo(LH, g), hi = t.node_hi(LH, g);
    const int64_t m = hi - lo;
    const int64_t pair0 = int64_t(pk.pairs.size());
    if (forward) {
      Pair p{};
      p.scale = 1.0f;
      p.f_off = pk.reserve_dev(m, m);
      p.in_buf = 0;
      p.in_row = lo;
      p.n = int32_t(m);
      p.lda = int32_t(m);
      pk.jobs->push_back({p.f_off, lo, int32_t(m), int32_t(pk.jobcols->size()), int32_t(m)});
      for (int32_t c = lo; c < hi; ++c) pk.jobcols->push_back(c);
      pk.table->push_back({0, LH, g, 0, 0, 0, 0, 0, m, m, p.f_off, m});
      if (pk.scales) pk.scales->push_back(1.0f);
      pk.pairs.push_back(p);
    }
    for (auto [k, a] : cover[size_t(g)]) {
      const Butterfly &bf = *bfs[size_t(k)];
      const Mat &last = bf.L == 0 ? bf.V0[0] : bf.W[bf.L][size_t(a)];
      const int64_t r = last.m;
      if (r == 0) continue;
      int64_t md[4];
      meta(bf, md);
      Pair p{};
      p.scale = 1.0f;
      p.in_buf = 1;
      p.in_row = int32_t(off[size_t(k)][bf.L][size_t(a)]);
      p.n = int32_t(r);
      p.lda = int32_t(m);
      if (forward) {
        const auto &sk = bf.bskel[size_t(a)];
        p.f_off = pk.reserve_dev(m, r);
        pk.jobs->push_back({p.f_off, lo, int32_t(m), int32_t(pk.jobcols->size()), int32_t(r)});
        pk.jobcols->insert(pk.jobcols->end(), sk.begin(), sk.end());
      } else {
        p.f_off = pk.put_host(bf.B[size_t(a)], &p.scale);
      }
      pk.table->push_back({3, md[0], md[1], md[2], md[3], bf.L, a, 0, m, r, p.f_off, m});
      if (pk.scales) pk.scales->push_back(p.scale);
      pk.pairs.push_back(p);
    }
    // one tile per kTileRows rows of the leaf, each with every pair (the first tile
    // uses the pairs above; later ones copies whose column-major blocks start r0 rows
    // further)
    const int64_t pair1 = int64_t(pk.pairs.size());
    if (pair1 == pair0) continue;
    for (int64_t r0 = 0; r0 < m; r0 += kTileRows) {
      Seg sg{};
      sg.m = int32_t(std::min<int64_t>(kTileRows, m - r0));
      sg.p0 = r0 == 0 ? int32_t(pair0) : int32_t(pk.pairs.size());
      if (r0 > 0)
        for (int64_t q = pair0; q < pair1; ++q) {
          Pair pr = pk.pairs[size_t(q)];
          pr.f_off += r0;
          pk.pairs.push_back(pr);
        }
      sg.p1 = r0 == 0 ? int32_t(pair1) : int32_t(pk.pairs.size());
      sg.map0 = int32_t(pk.rowmap.size());
      pk.rowmap.push_back({0, int32_t(lo + r0)});
      sg.map1 = int32_t(pk.rowmap.size());
      pk.segs.push_back(sg);
    }
  }
  const int64_t ns = int64_t(pk.segs.size()) - seg0;
  if (ns > 0) pk.launches.push_back({seg0, ns, final_beta, 1});
}

namespace {

Mat transposed(const Mat &f) {
  Mat t;
  t.m = f.n;
  t.n = f.m;
  t.v.resize(f.v.size());
  for (int k = 0; k < f.n; ++k)
    for (int i = 0; i < f.m; ++i) t.v[size_t(i) * f.n + k] = f.v[size_t(k) * f.m + i];
  return t;
}

// Tiles of at most kTileRows rows over an output block of `rows` rows at out_row of the
// destination: every tile sums all the pairs (column-major factors: a tile's rows start
// r0 further).
void emit_sum(PackSink &pk, const std::vector<Pair> &pairs, int64_t out_row, int64_t rows) {
  if (pairs.empty() || rows == 0) return;
  for (int64_t r0 = 0; r0 < rows; r0 += kTileRows) {
    Seg sg{};
    sg.m = int32_t(std::min<int64_t>(kTileRows, rows - r0));
    sg.p0 = int32_t(pk.pairs.size());
    for (Pair p : pairs) {
      p.f_off += r0;
      pk.pairs.push_back(p);
    }
    sg.p1 = int32_t(pk.pairs.size());
    sg.map0 = int32_t(pk.rowmap.size());
    pk.rowmap.push_back({0, int32_t(out_row + r0)});
    sg.map1 = int32_t(pk.rowmap.size());
    pk.segs.push_back(sg);
  }
}

}  // namespace

// The transposed product y = M^T x of a set of butterflies sharing their level count:
// the stages of pack_group in reverse with every factor transposed.  B^T blocks that
// read the same row leaf are stacked; a transposed transfer stage sums the two
// children's W^T contributions into one parent segment; the last launch sums the V^0
// blocks of every butterfly reading a column leaf into its output rows (beta 0:
// uncovered rows are left untouched).
void pack_group_t(PackSink &pk, const Tree &t, const std::vector<const Butterfly *> &bfs) {
  if (bfs.empty()) return;
  const int L = bfs[0]->L, ll = bfs[0]->hod_level + L;
  for (auto *bf : bfs)
    if (bf->L != L || bf->hod_level + bf->L != ll)
      fail(HODBF_E_ARG, "a transposed program needs butterflies of one shape");
  const int64_t nl = int64_t(1) << L;
  // outputs of forward stage s are the inputs of transposed step L - s; rows in T
  std::vector<std::vector<std::vector<int64_t>>> off(bfs.size(), std::vector<std::vector<int64_t>>(size_t(L + 1)));
  auto stage_rank = [&](const Butterfly &bf, int s, int64_t idx) {
    return s == 0 ? bf.V0[size_t(idx)].m : bf.W[size_t(s)][size_t(idx)].m;
  };
  for (int s = L; s >= 0; --s)
    for (size_t k = 0; k < bfs.size(); ++k) {
      const int64_t cnt = nl;  // 2^s x 2^(L - s) blocks at every stage
      off[k][size_t(s)].resize(size_t(cnt));
      for (int64_t e = 0; e < cnt; ++e) {
        off[k][size_t(s)][size_t(e)] = pk.t_rows;
        pk.t_rows += stage_rank(*bfs[k], s, e);
      }
    }
  // step 0: t(L, a) = B_a^T x(row leaf a), stacked by row leaf
  {
    const int64_t seg0 = int64_t(pk.segs.size());
    std::map<int64_t, std::vector<std::pair<size_t, int64_t>>> byleaf;
    for (size_t k = 0; k < bfs.size(); ++k)
      for (int64_t a = 0; a < nl; ++a)
        if (bfs[k]->B[size_t(a)].n > 0) byleaf[(bfs[k]->oi << L) + a].push_back({k, a});
    std::vector<Mat> keep;
    for (auto &[g, mem] : byleaf) {
      std::vector<Member> ms;
      keep.clear();
      keep.reserve(mem.size());
      for (auto [k, a] : mem) keep.push_back(transposed(bfs[k]->B[size_t(a)]));
      for (size_t q = 0; q < mem.size(); ++q)
        ms.push_back({&keep[q], off[mem[q].first][size_t(L)][size_t(mem[q].second)], 3, {0, 0, 0, 0}, L,
                      mem[q].second, 0});
      emit_group(pk, ms, 0, t.node_lo(ll, g), t.node_hi(ll, g) - t.node_lo(ll, g));
    }
    const int64_t ns = int64_t(pk.segs.size()) - seg0;
    if (ns > 0) pk.launches.push_back({seg0, ns, 0, 0});
  }
  // steps for s = L .. 1: t(s-1, (ap, 2b)) ++ t(s-1, (ap, 2b+1)) = sum_c W_{2ap+c, b}^T t(s, .)
  for (int s = L; s >= 1; --s) {
    const int64_t seg0 = int64_t(pk.segs.size());
    const int64_t nb = int64_t(1) << (L - s);
    for (size_t k = 0; k < bfs.size(); ++k) {
      const Butterfly &bf = *bfs[k];
      for (int64_t ap = 0; ap < (int64_t(1) << (s - 1)); ++ap)
        for (int64_t b = 0; b < nb; ++b) {
          const int64_t e0 = ap * 2 * nb + 2 * b;
          const int64_t rows = stage_rank(bf, s - 1, e0) + stage_rank(bf, s - 1, e0 + 1);
          if (rows == 0) continue;
          std::vector<Pair> prs;
          for (int c = 0; c < 2; ++c) {
            const int64_t e = (2 * ap + c) * nb + b;
            const Mat &W = bf.W[size_t(s)][size_t(e)];
            if (W.m == 0 || W.n == 0) continue;
            if (W.n != rows) fail(HODBF_E_ARG, "inconsistent transfer block");
            Pair p{};
            p.scale = 1.0f;
            p.f_off = pk.put_host(transposed(W), &p.scale);
            p.in_buf = 1;
            p.in_row = int32_t(off[k][size_t(s)][size_t(e)]);
            p.n = W.m;
            p.lda = int32_t(rows);
            prs.push_back(p);
          }
          emit_sum(pk, prs, off[k][size_t(s - 1)][size_t(e0)], rows);
        }
    }
    const int64_t ns = int64_t(pk.segs.size()) - seg0;
    if (ns > 0) pk.launches.push_back({seg0, ns, 0, 0});
  }
  // last step: y(column leaf) = sum over butterflies of V0_b^T t(0, b)
  {
    const int64_t seg0 = int64_t(pk.segs.size());
    std::map<int64_t, std::vector<std::pair<size_t, int64_t>>> byleaf;
    for (size_t k = 0; k < bfs.size(); ++k)
      for (int64_t b = 0; b < nl; ++b)
        if (bfs[k]->V0[size_t(b)].m > 0) byleaf[(bfs[k]->si << L) + b].push_back({k, b});
    for (auto &[g, mem] : byleaf) {
      const int32_t lo = t.node_lo(ll, g), hi = t.node_hi(ll, g);
      std::vector<Pair> prs;
      for (auto [k, b] : mem) {
        const Mat &V = bfs[k]->V0[size_t(b)];
        Pair p{};
        p.scale = 1.0f;
        p.f_off = pk.put_host(transposed(V), &p.scale);
        p.in_buf = 1;
        p.in_row = int32_t(off[k][0][size_t(b)]);
        p.n = V.m;
        p.lda = hi - lo;
        prs.push_back(p);
      }
      emit_sum(pk, prs, lo, hi - lo);
    }
    const int64_t ns = int64_t(pk.segs.size()) - seg0;
    if (ns > 0) pk.launches.push_back({seg0, ns, 0, 1});
  }
}

void check_program(const PackSink &pk, int64_t n_x, int64_t arena_count) {
  for (const Launch &ln : pk.launches) {
    const int64_t out_rows = ln.out ? n_x : pk.t_rows;
    for (int64_t s = ln.s0; s < ln.s0 + ln.ns; ++s) {
      const Seg &sg = pk.segs[size_t(s)];
      if (sg.m < 0 || sg.m > kTileRows || sg.p0 < 0 || sg.p1 < sg.p0 ||
          sg.p1 > int32_t(pk.pairs.size()) || sg.map0 < 0 || sg.map1 <= sg.map0 ||
          sg.map1 - sg.map0 > kMaxMapEntries || sg.map1 > int32_t(pk.rowmap.size()))
        fail(HODBF_E_ARG, "program check: malformed tile");
      for (int32_t p = sg.p0; p < sg.p1; ++p) {
        const Pair &pr = pk.pairs[size_t(p)];
        const int64_t in_rows = pr.in_buf ? pk.t_rows : n_x;
        if (pr.n < 0 || pr.in_row < 0 || int64_t(pr.in_row) + pr.n > in_rows)
          fail(HODBF_E_ARG, "program check: input rows out of range");
        if (pr.n > 0 && (pr.lda < sg.m || pr.f_off < 0 ||
                         (arena_count >= 0 && pr.f_off + int64_t(pr.n - 1) * pr.lda + sg.m > arena_count)))
          fail(HODBF_E_ARG, "program check: factor block out of range");
      }
      for (int32_t e = sg.map0; e < sg.map1; ++e) {
        const RowMap &rm = pk.rowmap[size_t(e)];
        const int32_t end = e + 1 < sg.map1 ? pk.rowmap[size_t(e + 1)].start : sg.m;
        if (rm.start < 0 || end < rm.start || end > sg.m || (e == sg.map0 && rm.start != 0) ||
            rm.out_row < 0 || int64_t(rm.out_row) + (end - rm.start) > out_rows)
          fail(HODBF_E_ARG, "program check: output rows out of range");
      }
    }
  }
}

void upload_program(Program &prog, PackSink &pk, hipStream_t st, bool log, int64_t n_x,
                    int64_t arena_count) {
  retile(pk, kRetileBelow, kTileRows / 2);
  if (n_x >= 0) check_program(pk, n_x, arena_count);
  for (Seg &sg : pk.segs)
    if (sg.p1 > sg.p0) sg.first = pk.pairs[size_t(sg.p0)];
  prog.io_rows = 0;
  for (const Launch &ln : pk.launches) {
    std::set<std::tuple<int32_t, int32_t, int32_t>> inputs;
    for (int64_t s = ln.s0; s < ln.s0 + ln.ns; ++s) {
      const Seg &sg = pk.segs[size_t(s)];
      prog.io_rows += sg.m;
      for (int32_t p = sg.p0; p < sg.p1; ++p) {
        const Pair &pr = pk.pairs[size_t(p)];
        inputs.insert({pr.in_buf, pr.in_row, pr.n});
      }
    }
    for (auto &in : inputs) prog.io_rows += std::get<2>(in);
  }
  // sort each launch's segments by row-tile count (their order within a launch is free:
  // they write disjoint rows) and record the class boundaries
  for (Launch &ln : pk.launches) {
    auto b = pk.segs.begin() + ln.s0, e = b + ln.ns;
    auto nrt = [](const Seg &sg) { return std::min(kRowClasses, std::max(1, (sg.m + 15) / 16)); };
    std::stable_sort(b, e, [&](const Seg &x, const Seg &y) { return nrt(x) < nrt(y); });
    for (int c = 0; c <= kRowClasses; ++c)
      ln.cls[c] = std::lower_bound(b, e, c + 1, [&](const Seg &sg, int v) { return nrt(sg) < v; }) - b;
  }
  // per-launch shape summary (tiles, rows, chunks of 16 columns per tile) for the log
  for (size_t li = 0; log && li < pk.launches.size(); ++li) {
    const Launch &ln = pk.launches[li];
    int64_t rows = 0, chunks = 0, cmax = 0;
    for (int64_t s = ln.s0; s < ln.s0 + ln.ns; ++s) {
      const Seg &sg = pk.segs[size_t(s)];
      int64_t c = 0;
      for (int32_t p = sg.p0; p < sg.p1; ++p) c += (pk.pairs[size_t(p)].n + 15) / 16;
      rows += sg.m;
      chunks += c;
      cmax = std::max(cmax, c);
    }
    logf("  launch %zu: %lld tiles, %.1f rows and %.1f chunks per tile, longest %lld chunks", li,
         (long long)ln.ns, ln.ns ? double(rows) / double(ln.ns) : 0.0,
         ln.ns ? double(chunks) / double(ln.ns) : 0.0, (long long)cmax);
  }
  prog.launches = pk.launches;
  prog.t_rows = pk.t_rows;
  prog.nseg = int64_t(pk.segs.size());
  prog.npair = int64_t(pk.pairs.size());
  if (prog.nseg) prog.segs.upload(pk.segs.data(), pk.segs.size() * sizeof(Seg), st);
  if (prog.npair) prog.pairs.upload(pk.pairs.data(), pk.pairs.size() * sizeof(Pair), st);
  // padded so a tile's kMaxMapEntries uniform reads stay inside the array
  pk.rowmap.resize(pk.rowmap.size() + kMaxMapEntries, RowMap{0, 0});
  prog.rowmap.upload(pk.rowmap.data(), pk.rowmap.size() * sizeof(RowMap), st);
}

}  // namespace hodbf
