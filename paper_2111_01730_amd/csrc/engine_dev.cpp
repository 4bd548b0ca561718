// Device engine of the preconditioner construction: multi-vectors in complex FP64 on
// the GPU, butterfly sets and dense diagonal blocks packed into grouped-GEMM programs
// (one forward, one transposed) over their own FP32 arena and run in FP64; elementwise
// work, sketch generation and row gathers by the kernels of construct.hip.  One stream
// throughout.
#include <map>

#include "construct.h"
#include "construct_dev.h"
#include "pack_sink.h"

namespace hodbf {

namespace {

class DevEngine;

struct DevMv final : Mv {
  DevEngine *eng = nullptr;
  DevBuf buf;
  double2 *p() const { return buf.as<double2>(); }
  ~DevMv() override;
};

const DevMv &dv(const Mv &m) { return static_cast<const DevMv &>(m); }
DevMv &dv(Mv &m) { return static_cast<DevMv &>(m); }

class DevEngine final : public Engine {
 public:
  DevEngine(const Tree *t, hipStream_t st, int mc) : st_(st), mc_(mc) { tree = t; }
  int max_cols() const override { return mc_; }
  hipStream_t stream() const { return st_; }

  MvP make(int R) override {
    auto m = std::make_shared<DevMv>();
    m->R = R;
    m->eng = this;
    const size_t bytes = size_t(n()) * size_t(R) * sizeof(double2);
    auto it = pool_.find(bytes);
    if (it != pool_.end()) {
      m->buf = std::move(it->second);
      pool_.erase(it);
    } else {
      m->buf.alloc(bytes);
    }
    // not cleared: every multi-vector of the construction is written whole by its
    // producer (a fill, a copy or an operator apply) before it is read
    return m;
  }
  void recycle(DevBuf &&b) {
    if (b.p) pool_.emplace(b.bytes, std::move(b));
  }
  void zero(Mv &y) override {
    if (dv(y).buf.bytes) HIPCHK(hipMemsetAsync(dv(y).buf.p, 0, dv(y).buf.bytes, st_));
  }
  void copy(const Mv &x, Mv &y) override {
    if (x.R != y.R) fail(HODBF_E_ARG, "multi-vector widths differ");
    if (&x != &y && dv(x).buf.bytes)
      HIPCHK(hipMemcpyAsync(dv(y).buf.p, dv(x).buf.p, dv(x).buf.bytes, hipMemcpyDeviceToDevice, st_));
  }
  void axpy(cd a, const Mv &x, Mv &y) override {
    if (x.R != y.R) fail(HODBF_E_ARG, "multi-vector widths differ");
    launch_axpy_c128(dv(y).p(), dv(x).p(), a.real(), a.imag(), n() * x.R, st_);
    HIPCHK(hipGetLastError());
  }
  void keep_rows(const RowSet &rows, Mv &y) override {
    // row masks recur (the same child row sets in every product of one recursion step):
    // kept on the device, keyed by their ranges
    auto it = masks_.find(rows);
    if (it == masks_.end()) {
      if (masks_.size() > 64) masks_.clear();
      std::vector<uint8_t> keep(size_t(n()), 0);
      for (auto [lo, hi] : rows)
        for (int32_t r = lo; r < hi; ++r) keep[size_t(r)] = 1;
      DevBuf b;
      b.upload(keep.data(), keep.size(), st_);
      it = masks_.emplace(rows, std::move(b)).first;
    }
    launch_keep_rows_c128(dv(y).p(), it->second.as<uint8_t>(), n(), y.R, st_);
    HIPCHK(hipGetLastError());
  }
  void fill_sketch(Mv &x, const std::vector<int32_t> &slot_of_row, int64_t col0, int k,
                   uint64_t seed) override {
    stage(slots_, slot_of_row.data(), slot_of_row.size() * sizeof(int32_t));
    launch_fill_sketch_c128(dv(x).p(), slots_.as<int32_t>(), n(), x.R, col0, k, seed, st_);
    HIPCHK(hipGetLastError());
  }
  void fill_unit(Mv &x, const std::vector<int32_t> &col_of_row) override {
    stage(slots_, col_of_row.data(), col_of_row.size() * sizeof(int32_t));
    launch_fill_unit_c128(dv(x).p(), slots_.as<int32_t>(), n(), x.R, st_);
    HIPCHK(hipGetLastError());
  }
  void gather(const Mv &y, const std::vector<Gather> &req, int k, std::vector<cd> &out) override {
    std::vector<int32_t> rows, q0;
    for (const Gather &g : req)
      for (int32_t r : g.rows) {
        if (r < 0 || r >= n() || g.q0 < 0 || g.q0 + k > y.R) fail(HODBF_E_ARG, "gather out of range");
        rows.push_back(r);
        q0.push_back(g.q0);
      }
    out.assign(rows.size() * size_t(k), cd(0, 0));
    if (rows.empty()) return;
    stage(grows_, rows.data(), rows.size() * sizeof(int32_t));
    stage(gq0_, q0.data(), q0.size() * sizeof(int32_t));
    grow(gout_, rows.size() * size_t(k) * sizeof(double2));
    launch_gather_rows_c128(dv(y).p(), y.R, grows_.as<int32_t>(), gq0_.as<int32_t>(),
                            int64_t(rows.size()), k, gout_.as<double2>(), st_);
    HIPCHK(hipGetLastError());
    std::vector<double2> h(rows.size() * size_t(k));
    HIPCHK(hipMemcpyAsync(h.data(), gout_.p, h.size() * sizeof(double2), hipMemcpyDeviceToHost, st_));
    HIPCHK(hipStreamSynchronize(st_));
    for (size_t i = 0; i < h.size(); ++i) out[i] = cd(h[i].x, h[i].y);
  }
  OpP butterflies(std::vector<Butterfly> bfs) override;
  OpP dense_diag(std::vector<DenseDiag> blocks) override;

  // program workspace, grown on demand (programs run one at a time on the stream)
  double2 *work(int64_t rows, int R) {
    grow(work_, size_t(std::max<int64_t>(rows, 1)) * size_t(R) * sizeof(double2));
    return work_.as<double2>();
  }

 private:
  // grow-only device buffers: an allocation (and the free before it) synchronizes the
  // device, so staging buffers are only ever enlarged
  static void grow(DevBuf &b, size_t bytes) {
    if (b.bytes < bytes) b.alloc(std::max(bytes, b.bytes + b.bytes / 4));
  }
  // copy host data into a staging buffer; the stream is synchronized so the caller's
  // host vector may go away
  void stage(DevBuf &b, const void *src, size_t bytes) {
    grow(b, bytes);
    if (bytes) {
      HIPCHK(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, st_));
      HIPCHK(hipStreamSynchronize(st_));
    }
  }

  hipStream_t st_;
  int mc_;
  std::multimap<size_t, DevBuf> pool_;
  std::map<RowSet, DevBuf> masks_;
  DevBuf work_, slots_, grows_, gq0_, gout_;
};

DevMv::~DevMv() {
  if (eng) eng->recycle(std::move(buf));
}

// A linear operator held as a forward and a transposed grouped-GEMM program over one
// complex FP32 arena; y is cleared first (the programs write covered rows only).
class DevProgOp final : public LinOp {
 public:
  DevBuf arena;
  Program fwd, trans;
  void apply(Engine &E, bool tr, const Mv &x, Mv &y) const override {
    DevEngine &D = static_cast<DevEngine &>(E);
    if (x.R != y.R) fail(HODBF_E_ARG, "multi-vector widths differ");
    D.zero(y);
    const Program &p = tr ? trans : fwd;
    if (p.launches.empty()) return;
    double2 *T = D.work(p.t_rows, x.R);
    for (const Launch &ln : p.launches)
      launch_grouped_f64(p.segs.as<Seg>(), p.pairs.as<Pair>(), p.rowmap.as<RowMap>(), ln.s0, ln.ns,
                         arena.as<float2>(), dv(x).p(), T, ln.out ? dv(y).p() : T, x.R, ln.beta,
                         D.stream());
    HIPCHK(hipGetLastError());
  }
};

struct HostArena {
  std::vector<float2> v;
  int64_t put(const Mat &f, float *scale) {
    *scale = 1.0f;
    const int64_t off = (int64_t(v.size()) + 15) & ~int64_t(15);
    v.resize(size_t(off + int64_t(f.m) * f.n), make_float2(0.f, 0.f));
    for (size_t e = 0; e < f.v.size(); ++e) v[size_t(off) + e] = make_float2(f.v[e].real(), f.v[e].imag());
    return off;
  }
};

OpP DevEngine::butterflies(std::vector<Butterfly> bfs) {
  auto op = std::make_shared<DevProgOp>();
  for (Butterfly &bf : bfs) prune_butterfly(bf);
  std::vector<const Butterfly *> ptrs;
  for (const Butterfly &bf : bfs) ptrs.push_back(&bf);
  HostArena ha;
  std::vector<BlockRec> table;
  std::vector<PackSink> packs;
  for (int dir = 0; dir < 2; ++dir) {
    PackSink pk;
    pk.table = &table;
    pk.put_host = [&](const Mat &f, float *scale) { return ha.put(f, scale); };
    if (dir == 0)
      pack_group(pk, *tree, ptrs, false, 0, [](const Butterfly &, int64_t *md) {
        md[0] = md[1] = md[2] = md[3] = 0;
      });
    else
      pack_group_t(pk, *tree, ptrs);
    check_program(pk, n(), -1);
    packs.push_back(std::move(pk));
  }
  for (int dir = 0; dir < 2; ++dir) {
    check_program(packs[size_t(dir)], n(), int64_t(ha.v.size()));
    upload_program(dir == 0 ? op->fwd : op->trans, packs[size_t(dir)], st_, false, n(),
                   int64_t(ha.v.size()));
  }
  if (!ha.v.empty()) op->arena.upload(ha.v.data(), ha.v.size() * sizeof(float2), st_);
  return op;
}

OpP DevEngine::dense_diag(std::vector<DenseDiag> blocks) {
  auto op = std::make_shared<DevProgOp>();
  HostArena ha;
  std::vector<PackSink> packs;
  for (int dir = 0; dir < 2; ++dir) {
    PackSink pk;
    for (const DenseDiag &d : blocks) {
      const int m = d.D.m;
      Mat T;
      const Mat *src = &d.D;
      if (dir == 1) {
        T.m = T.n = m;
        T.v.resize(d.D.v.size());
        for (int k = 0; k < m; ++k)
          for (int i = 0; i < m; ++i) T.v[size_t(i) * m + k] = d.D.v[size_t(k) * m + i];
        src = &T;
      }
      float scale = 1.0f;
      const int64_t off = ha.put(*src, &scale);
      for (int r0 = 0; r0 < m; r0 += kTileRows) {
        Pair pr{};
        pr.f_off = off + r0;
        pr.in_row = d.lo;
        pr.n = m;
        pr.lda = m;
        pr.in_buf = 0;
        pr.scale = 1.0f;
        Seg sg{};
        sg.m = std::min(kTileRows, m - r0);
        sg.p0 = int32_t(pk.pairs.size());
        sg.p1 = sg.p0 + 1;
        sg.map0 = int32_t(pk.rowmap.size());
        sg.map1 = sg.map0 + 1;
        pk.rowmap.push_back({0, d.lo + r0});
        pk.pairs.push_back(pr);
        pk.segs.push_back(sg);
      }
    }
    if (!pk.segs.empty()) pk.launches.push_back({0, int64_t(pk.segs.size()), 0, 1});
    packs.push_back(std::move(pk));
  }
  for (int dir = 0; dir < 2; ++dir) {
    check_program(packs[size_t(dir)], n(), int64_t(ha.v.size()));
    upload_program(dir == 0 ? op->fwd : op->trans, packs[size_t(dir)], st_, false, n(),
                   int64_t(ha.v.size()));
  }
  if (!ha.v.empty()) op->arena.upload(ha.v.data(), ha.v.size() * sizeof(float2), st_);
  return op;
}

}  // namespace

std::unique_ptr<Engine> make_device_engine(const Tree *t, hipStream_t st, int max_cols) {
  return std::make_unique<DevEngine>(t, st, max_cols);
}

}  // namespace hodbf
