// Packing of butterfly factors into device programs: stage-by-stage grouped launches
// (all butterflies of a set advance one level per launch) and a final per-leaf reduce
// that applies the outer factors B^L (and the dense leaf blocks for Z_con).
#include <algorithm>
#include <functional>

#include "pack_sink.h"

namespace hodbf {

namespace {
constexpr int kTile = 64;  // output rows per segment (4 MFMA row tiles)
}



static void add_seg(PackSink &pk, int64_t out_row, int64_t m, const std::vector<Pair> &prs) {
  // prs all share m rows; split rows into tiles of kTile
  for (int64_t i0 = 0; i0 < m; i0 += kTile) {
    Seg s;
    s.out_row = int32_t(out_row + i0);
    s.m = int32_t(std::min<int64_t>(kTile, m - i0));
    s.p0 = int32_t(pk.pairs.size());
    for (Pair p : prs) {
      p.f_off += i0;
      pk.pairs.push_back(p);
    }
    s.p1 = int32_t(pk.pairs.size());
    pk.segs.push_back(s);
  }
}

// Pack one set of butterflies whose row and column trees end at the leaves of T_H.
// meta(bf) gives (l, i, ca, cb) for the block table.
void pack_group(PackSink &pk, const Tree &t, const std::vector<const Butterfly *> &bfs,
                bool forward, int final_beta,
                const std::function<void(const Butterfly &, int64_t *)> &meta) {
  const int LH = t.depth;
  int Lmax = -1;
  for (auto *bf : bfs) Lmax = std::max(Lmax, bf->L);
  // off[k][s][idx]: first workspace row of output (a, b) at stage s of butterfly k
  std::vector<std::vector<std::vector<int64_t>>> off(bfs.size());
  for (size_t k = 0; k < bfs.size(); ++k) off[k].resize(bfs[k]->L + 1);
  for (int s = 0; s <= Lmax; ++s) {
    const int64_t seg0 = int64_t(pk.segs.size());
    for (size_t k = 0; k < bfs.size(); ++k) {
      const Butterfly &bf = *bfs[k];
      if (bf.L < s) continue;
      const int64_t na = int64_t(1) << s, nb = int64_t(1) << (bf.L - s);
      int64_t md[4];
      meta(bf, md);
      off[k][s].resize(static_cast<size_t>(na * nb));
      for (int64_t a = 0; a < na; ++a)
        for (int64_t b = 0; b < nb; ++b) {
          const Mat &f = s == 0 ? bf.V0[size_t(b)] : bf.W[s][size_t(a * nb + b)];
          const int64_t out_row = pk.t_rows;
          off[k][s][size_t(a * nb + b)] = out_row;
          pk.t_rows += f.m;
          if (f.m == 0 || f.n == 0) continue;
          Pair p{};
          p.lda = f.m;
          p.n = f.n;
          if (s == 0) {
            const int64_t nu = (bf.si << bf.L) + b;
            p.in_buf = 0;
            p.in_row = t.node_lo(LH, nu);
          } else {
            p.in_buf = 1;
            p.in_row = int32_t(off[k][s - 1][size_t((a / 2) * 2 * nb + 2 * b)]);
          }
          p.f_off = pk.put_host(f, &p.scale);
          pk.table->push_back({s == 0 ? 1 : 2, md[0], md[1], md[2], md[3], s, a, b, f.m, f.n,
                               p.f_off});
          if (pk.scales) pk.scales->push_back(p.scale);
          add_seg(pk, out_row, f.m, {p});
        }
    }
    const int64_t ns = int64_t(pk.segs.size()) - seg0;
    if (ns > 0) pk.launches.push_back({seg0, ns, 0, 0});
  }
  // final reduce: every leaf g gets its dense block (forward) and one outer block B_a
  // from each butterfly whose row tree holds g
  const int64_t nleaf = int64_t(1) << LH;
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
    std::vector<Pair> prs;
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
      pk.table->push_back({0, LH, g, 0, 0, 0, 0, 0, m, m, p.f_off});
      if (pk.scales) pk.scales->push_back(1.0f);
      prs.push_back(p);
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
      pk.table->push_back({3, md[0], md[1], md[2], md[3], bf.L, a, 0, m, r, p.f_off});
      if (pk.scales) pk.scales->push_back(p.scale);
      prs.push_back(p);
    }
    if (!prs.empty()) add_seg(pk, lo, m, prs);
  }
  const int64_t ns = int64_t(pk.segs.size()) - seg0;
  if (ns > 0) pk.launches.push_back({seg0, ns, final_beta, 1});
}

void upload_program(Program &prog, PackSink &pk, hipStream_t st) {
  prog.launches = pk.launches;
  prog.t_rows = pk.t_rows;
  prog.nseg = int64_t(pk.segs.size());
  prog.npair = int64_t(pk.pairs.size());
  if (prog.nseg) prog.segs.upload(pk.segs.data(), pk.segs.size() * sizeof(Seg), st);
  if (prog.npair) prog.pairs.upload(pk.pairs.data(), pk.pairs.size() * sizeof(Pair), st);
}

}  // namespace hodbf
