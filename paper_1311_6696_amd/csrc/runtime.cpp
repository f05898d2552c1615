// Host runtime: pool, views, recorder.
#include "runtime.hpp"

#include <algorithm>
#include <climits>

namespace pe {

// ------------------------------------------------------------------ Pool ----
static size_t size_class(size_t b) {
  if (b < 256) return 256;
  size_t p = 1;
  while (p < b) p <<= 1;
  if (p <= (size_t(1) << 20)) return p;
  const size_t step = p >> 3;   // 1/8 steps above 1 MiB
  return (b + step - 1) / step * step;
}

Pool::~Pool() {
  for (auto& kv : free_)
    for (void* p : kv.second) dev::free(p);
  for (auto& kv : size_of_) (void)kv;   // blocks still in use are leaked deliberately
}

void* Pool::alloc(size_t bytes) {
  const size_t sc = size_class(bytes);
  auto it = free_.find(sc);
  void* p;
  if (it != free_.end() && !it->second.empty()) {
    p = it->second.back();
    it->second.pop_back();
  } else {
    try {
      p = dev::malloc(sc);
    } catch (const Error&) {
      trim();
      p = dev::malloc(sc);
    }
    size_of_[p] = sc;
  }
  in_use_ += sc;
  return p;
}

void Pool::release(void* p) {
  if (!p) return;
  auto it = size_of_.find(p);
  if (it == size_of_.end()) return;
  in_use_ -= it->second;
  free_[it->second].push_back(p);
}

void Pool::trim() {
  for (auto& kv : free_)
    for (void* p : kv.second) {
      size_of_.erase(p);
      dev::free(p);
    }
  free_.clear();
}

void Ctx::clear_graphs() {
  for (auto& kv : graph_cache)
    for (Graph& g : kv.second) {
      dev::graph_destroy(g.exec);
      pool.release(g.dblob);
      pool.release(g.partials);
      pool.release(g.counters);
    }
  graph_cache.clear();
  graph_count = 0;
}

Ctx::~Ctx() {
  clear_graphs();
  dev::stream_destroy(capture_stream);
  for (auto& p : pinned_free) dev::host_free(p.second);
}

void* Ctx::pinned_get(size_t bytes) {
  auto it = pinned_free.lower_bound(bytes);
  if (it != pinned_free.end()) {
    void* p = it->second;
    pinned_free.erase(it);
    return p;
  }
  size_t cap = 1 << 16;
  while (cap < bytes) cap <<= 1;
  void* p = dev::host_alloc(cap);
  pinned_size[p] = cap;
  return p;
}

void Ctx::pinned_put(void* p, size_t) { pinned_free.emplace(pinned_size[p], p); }

// ----------------------------------------------------------------- views ----
TV dense(const void* p, int dt, const std::string& idx, const Dims& dims) {
  PE_REQUIRE(idx.size() == dims.size(), "view rank mismatch for '" + idx + "'");
  TV v;
  v.p = p;
  v.dt = dt;
  v.idx = idx;
  v.dim = dims;
  v.str.assign(dims.size(), 0);
  int64_t s = 1;
  for (int i = (int)dims.size() - 1; i >= 0; --i) {
    v.str[i] = s;
    s *= dims[i];
  }
  return v;
}

TV relabel(TV v, const std::string& idx) {
  PE_REQUIRE(idx.size() == v.idx.size(), "relabel rank mismatch");
  v.idx = idx;
  return v;
}

namespace {
struct Sub {
  int64_t dim, s1, s2;
};
using Subs = SmallVec<Sub, 16>;
void merge_subs(Subs& v) {
  Subs out;
  for (const Sub& s : v) {
    if (!out.empty() && out.back().s1 == s.s1 * s.dim && out.back().s2 == s.s2 * s.dim) {
      out.back().dim *= s.dim;
      out.back().s1 = s.s1;
      out.back().s2 = s.s2;
    } else {
      out.push_back(s);
    }
  }
  if (out.empty()) out.push_back({1, 0, 0});
  v = out;
}
int find_idx(const TV& t, char c) {
  const char* s = t.idx.data();
  const int n = (int)t.idx.size();
  for (int i = 0; i < n; ++i)
    if (s[i] == c) return i;
  return -1;
}
}  // namespace

TcDesc tc_build(const TV& C, const TV& X, const TV& Y, double alpha, double beta) {
  // Operand "A" is the one holding C's unit-stride index, so that the MFMA
  // tile's contiguous lane group writes contiguous memory.
  char cin = 0;
  int64_t best = INT64_MAX;
  for (size_t i = 0; i < C.idx.size(); ++i)
    if (C.dim[i] > 1 && C.str[i] < best) {
      best = C.str[i];
      cin = C.idx[i];
    }
  const bool x_is_a = (cin == 0) || find_idx(X, cin) >= 0;
  const TV& A = x_is_a ? X : Y;
  const TV& B = x_is_a ? Y : X;
  Subs Ms, Ns, Ks;
  for (size_t i = 0; i < C.idx.size(); ++i) {
    const char c = C.idx[i];
    const int ia = find_idx(A, c), ib = find_idx(B, c);
    if (ia < 0 && ib < 0 && C.dim[i] == 1) continue;   // trivial index of the output only
    PE_REQUIRE((ia >= 0) != (ib >= 0), std::string("index '") + c + "' must be in exactly one operand");
    if (ia >= 0) {
      PE_REQUIRE(A.dim[ia] == C.dim[i], std::string("dimension mismatch of '") + c + "'");
      if (C.dim[i] > 1) Ms.push_back({C.dim[i], A.str[ia], C.str[i]});
    } else {
      PE_REQUIRE(B.dim[ib] == C.dim[i], std::string("dimension mismatch of '") + c + "'");
      if (C.dim[i] > 1) Ns.push_back({C.dim[i], B.str[ib], C.str[i]});
    }
  }
  for (size_t i = 0; i < A.idx.size(); ++i) {
    const char c = A.idx[i];
    if (find_idx(C, c) >= 0) continue;
    const int ib = find_idx(B, c);
    if (ib < 0 && A.dim[i] == 1) continue;
    PE_REQUIRE(ib >= 0, std::string("index '") + c + "' appears once");
    PE_REQUIRE(B.dim[ib] == A.dim[i], std::string("dimension mismatch of '") + c + "'");
    if (A.dim[i] > 1) Ks.push_back({A.dim[i], A.str[i], B.str[ib]});
  }
  for (size_t i = 0; i < B.idx.size(); ++i)
    PE_REQUIRE(find_idx(C, B.idx[i]) >= 0 || find_idx(A, B.idx[i]) >= 0 || B.dim[i] == 1,
               std::string("index '") + B.idx[i] + "' appears once");
  merge_subs(Ms);
  merge_subs(Ns);
  merge_subs(Ks);
  PE_REQUIRE(Ms.size() <= TC_MAXD && Ns.size() <= TC_MAXD && Ks.size() <= TC_MAXD,
             "contraction " + C.idx + " = " + X.idx + " * " + Y.idx + " needs more than 4 sub-dimensions");
  TcDesc d;
  std::memset(&d, 0, sizeof(d));
  d.A = A.p;
  d.B = B.p;
  d.C = const_cast<void*>(C.p);
  int64_t M = 1, N = 1, K = 1;
  d.nm = (int)Ms.size();
  d.nn = (int)Ns.size();
  d.nk = (int)Ks.size();
  for (int i = 0; i < d.nm; ++i) {
    d.dm[i] = (int32_t)Ms[i].dim;
    d.sAm[i] = Ms[i].s1;
    d.sCm[i] = Ms[i].s2;
    M *= Ms[i].dim;
  }
  for (int i = 0; i < d.nn; ++i) {
    d.dn[i] = (int32_t)Ns[i].dim;
    d.sBn[i] = Ns[i].s1;
    d.sCn[i] = Ns[i].s2;
    N *= Ns[i].dim;
  }
  for (int i = 0; i < d.nk; ++i) {
    d.dk[i] = (int32_t)Ks[i].dim;
    d.sAk[i] = Ks[i].s1;
    d.sBk[i] = Ks[i].s2;
    K *= Ks[i].dim;
  }
  PE_REQUIRE(M < INT_MAX && N < INT_MAX && K < INT_MAX, "contraction too large");
  d.M = (int)M;
  d.N = (int)N;
  d.K = (int)K;
  // load along k when k, not the output index, is unit-stride in the operand
  const bool k_unit_a = !Ks.empty() && Ks.back().s1 == 1, k_unit_b = !Ks.empty() && Ks.back().s2 == 1;
  d.a_kfast = (k_unit_a && (Ms.empty() || Ms.back().s1 != 1)) ? 1 : 0;
  d.b_kfast = (k_unit_b && (Ns.empty() || Ns.back().s1 != 1)) ? 1 : 0;
  d.alpha = alpha;
  d.beta = beta;
  return d;
}

// Fused ket-bra descriptor from labelled views: every label of the four
// views lies in exactly two of them, which fixes its group.  Sub-dimensions
// of a group follow the label order of the view named last (R and the
// output groups follow Y, so R ends with Y's unit-stride index).
KbDesc kb_build(const TV& Y, const TV& X, const TV& K, const TV& B) {
  KbDesc d;
  std::memset(&d, 0, sizeof(d));
  d.X = X.p;
  d.K = K.p;
  d.B = B.p;
  d.Y = const_cast<void*>(Y.p);
  auto group = [](KbGroup& g, const TV& t0, const TV& t1, const TV& order, const TV& excl1, const TV& excl2) {
    Subs subs;
    for (size_t i = 0; i < order.idx.size(); ++i) {
      const char c = order.idx[i];
      const int i0 = find_idx(t0, c), i1 = find_idx(t1, c);
      if (i0 < 0 || i1 < 0) continue;
      PE_REQUIRE(find_idx(excl1, c) < 0 && find_idx(excl2, c) < 0, std::string("index '") + c + "' in three views");
      PE_REQUIRE(t0.dim[i0] == t1.dim[i1], std::string("dimension mismatch of '") + c + "'");
      if (t0.dim[i0] > 1) subs.push_back({t0.dim[i0], t0.str[i0], t1.str[i1]});
    }
    merge_subs(subs);
    PE_REQUIRE(subs.size() <= (size_t)KB_MAXD, "fused contraction group with more than 4 sub-dimensions");
    g.n = (int)subs.size();
    int64_t size = 1;
    for (int j = 0; j < g.n; ++j) {
      g.dim[j] = (int32_t)subs[j].dim;
      g.s0[j] = subs[j].s1;
      g.s1[j] = subs[j].s2;
      size *= subs[j].dim;
    }
    PE_REQUIRE(size < INT_MAX, "fused contraction too large");
    g.size = (int32_t)size;
  };
  group(d.r, X, Y, Y, K, B);
  group(d.lu, X, K, K, Y, B);
  group(d.q, X, B, B, Y, K);
  group(d.p, K, B, K, X, Y);
  group(d.dr, K, Y, Y, X, B);
  group(d.gs, B, Y, Y, X, K);
  // every label lies in two views
  for (const TV* t : {&X, &K, &B, &Y})
    for (size_t i = 0; i < t->idx.size(); ++i) {
      const char c = t->idx[i];
      const int n = (find_idx(X, c) >= 0) + (find_idx(K, c) >= 0) + (find_idx(B, c) >= 0) + (find_idx(Y, c) >= 0);
      PE_REQUIRE(n == 2 || t->dim[i] == 1, std::string("index '") + c + "' must be in exactly two views");
    }
  return d;
}

// The fused kernel pays off for long R (the two-row sandwiches); for short
// R (ALS site steps) its per-block serial phases cost more latency than the
// two separate launches.
bool kb_fits(const KbDesc& d, int prec) {
  if (prec == TP_BF16 || d.r.size < 1024) return false;
  if (d.r.n < 1 || d.r.s0[d.r.n - 1] != 1 || d.r.s1[d.r.n - 1] != 1) return false;
  if (d.dr.size * d.p.size > 32 || d.p.size > 2 || d.gs.size > 16 || d.dr.size > 16 || d.lu.size > 64) return false;
  const int nb1 = d.dr.size * d.p.size > 16 ? 2 : 1;
  const int lup = (d.lu.size + 3) / 4 * 4, pqp = (d.p.size * d.q.size + 3) / 4 * 4;
  return kb_lds_bytes(prec, nb1, lup, pqp, d.q.size) <= 64 * 1024;
}

double kb_flops(const KbDesc& d) {
  const double r = d.r.size, lu = d.lu.size, q = d.q.size, p = d.p.size, dr = d.dr.size, gs = d.gs.size;
  return 2.0 * r * lu * q * dr * p + 2.0 * r * dr * p * q * gs;
}

// -------------------------------------------------------------- recorder ----
enum OpKind { OK_TC = 0, OK_QR = 1, OK_RED = 2, OK_EW = 3, OK_SEP = 4, OK_TCR = 5, OK_TCS = 6, OK_KB = 7, OK_K2 = 8, OK_CQ = 9, OK_KC = 10, OK_TSK = 11 };

size_t Rec::push_bytes(const void* p, size_t n) {
  const size_t off = (blob_.size() + 15) / 16 * 16;
  blob_.resize(off);
  blob_.insert(blob_.end(), (const uint8_t*)p, (const uint8_t*)p + n);
  return off;
}

// Tile family of one contraction: skinny outputs (N <= 16, N <= 32), short
// M, outputs whose width fits 48 or 80 columns (dD^2-type legs, little
// padding), or general.  A grouped launch runs one tile shape, so a group is
// split by family before the shape is chosen.
static int tile_family(const TcDesc& d) {
  if (d.N <= 16) return 0;
  if (d.N <= 32) return 1;
  if (d.M <= 32) return 2;
  if (d.N <= 48) return 3;
  if (d.N > 64 && d.N <= 80) return 4;
  return 5;
}
constexpr int N_FAMILIES = 6;

// Largest tile of the family that still gives two workgroups per CU.
static int pick_tile(int family, const std::vector<TcDesc>& ds) {
  static const std::vector<int> CAND[N_FAMILIES] = {{TT_256x16, TT_64x16}, {TT_128x32, TT_64x32}, {TT_32x128},
                                                    {TT_128x48, TT_64x32}, {TT_64x80, TT_64x32},
                                                    {TT_64x64, TT_64x32}};
  const std::vector<int>& cand = CAND[family];
  constexpr int64_t WANT = 2 * 256;
  for (int t : cand) {
    int64_t tiles = 0;
    for (const auto& d : ds)
      tiles += (int64_t)((d.M + tile_mt(t) - 1) / tile_mt(t)) * ((d.N + tile_nt(t) - 1) / tile_nt(t));
    if (tiles >= WANT) return t;
  }
  return cand.back();
}

// Algorithmic bytes of one contraction: A and B read once, C written once
// (and read when accumulated), in the operand and output element sizes.
static double tc_bytes(int prec, int out_dt, const TcDesc& d) {
  const double es = prec == TP_F64 ? 8.0 : 4.0, os = out_dt == DT_F64 ? 8.0 : 4.0;
  return es * ((double)d.M * d.K + (double)d.K * d.N) + os * (double)d.M * d.N * (d.beta != 0.0 ? 2.0 : 1.0);
}

// Contractions the skinny kernel can take: outputs at most 80 wide, K at
// most 128 (B staged in shared memory), m unit-stride in A and C.
static bool skinny_fits(const TcDesc& d) {
  return d.N <= 80 && d.K <= 128 && d.sAm[d.nm - 1] == 1 && d.sCm[d.nm - 1] == 1;
}

// Launch shapes of one group: the skinny kernel, or a tile with the split-K
// rule on (code = tile) or off (code = NO_SPLIT + tile).  HEURISTIC: the
// skinny kernel when the group qualifies, else the family's tile.
enum : int { HEURISTIC = -1, SKINNY = 1000, NO_SPLIT = 100 };

// Signature of a group for the tuned-choice table: precision, output type,
// family, skinny eligibility, widest N, longest K, total rows and group
// size (both to the next power of two).
static uint64_t tune_key(int prec, int out_dt, int fam, bool skinny, const std::vector<TcDesc>& ds) {
  int64_t rows = 0;
  int maxN = 0, maxK = 0;
  for (const auto& d : ds) {
    rows += d.M;
    maxN = std::max(maxN, d.N);
    maxK = std::max(maxK, d.K);
  }
  int lr = 0, ld = 0;
  while ((int64_t(1) << lr) < rows) ++lr;
  while ((1 << ld) < (int)ds.size()) ++ld;
  uint64_t k = (uint64_t)prec;
  k = k * 2 + (uint64_t)out_dt;
  k = k * 8 + (uint64_t)fam;
  k = k * 2 + (skinny ? 1 : 0);
  k = k * 65536 + (uint64_t)std::min(maxN, 65535);
  k = k * 65536 + (uint64_t)std::min(maxK, 65535);
  k = k * 64 + (uint64_t)lr;
  k = k * 32 + (uint64_t)ld;
  return k;
}

// A contraction the short skinny kernel takes: FP64 with beta = 0, one
// sub-dimension per index group, the narrow output side (<= 32) as n (the
// operands swap roles when it is m), the wide side <= 4096, 128 <= K <= 8192.
static bool tsk_from(const TcDesc& d, TskDesc& t) {
  if (d.nm != 1 || d.nn != 1 || d.nk != 1 || d.beta != 0.0 || d.K < 128 || d.K > 8192) return false;
  const bool swap = d.N > 32;
  const int M = swap ? d.N : d.M, N = swap ? d.M : d.N;
  if (N > 32 || M > 4096) return false;
  std::memset(&t, 0, sizeof(t));
  if (!swap) {
    t.A = (const double*)d.A;
    t.sAm = d.sAm[0];
    t.sAk = d.sAk[0];
    t.B = (const double*)d.B;
    t.sBk = d.sBk[0];
    t.sBn = d.sBn[0];
    t.sCm = d.sCm[0];
    t.sCn = d.sCn[0];
  } else {   // C^T = B^T A^T
    t.A = (const double*)d.B;
    t.sAm = d.sBn[0];
    t.sAk = d.sBk[0];
    t.B = (const double*)d.A;
    t.sBk = d.sAk[0];
    t.sBn = d.sAm[0];
    t.sCm = d.sCn[0];
    t.sCn = d.sCm[0];
  }
  t.C = (double*)d.C;
  t.M = M;
  t.N = N;
  t.K = d.K;
  t.alpha = d.alpha;
  return true;
}

void Rec::tsk(std::vector<TskDesc> ds, bool algorithmic) {
  if (ds.empty()) return;
  int64_t blocks = 0, parts = 0;
  double fl = 0.0, by = 0.0;
  for (auto& t : ds) {
    const int tiles = (t.M + TSK_MT - 1) / TSK_MT;
    t.ksplit = (t.K + TSK_KS - 1) / TSK_KS;
    t.tile_base = (int32_t)blocks;
    blocks += (int64_t)tiles * t.ksplit;
    t.cnt_base = cq_slots_;
    cq_slots_ += tiles;
    parts += (int64_t)tiles * t.ksplit * TSK_MT * 32;
    fl += 2.0 * t.M * (double)t.N * t.K;
    by += 8.0 * ((double)t.M * t.K + (double)t.K * t.N + (double)t.M * t.N);
  }
  PE_REQUIRE(blocks < INT_MAX, "too many tiles in one launch");
  // the partial buffer is shared with the split-K contractions: launches run
  // in stream order and each finishes its sums before the next starts
  if ((size_t)parts > part_cap_) {
    part_cap_ = std::max((size_t)parts, part_cap_ * 2);
    part_buf_ = (double*)scratch_->alloc(sizeof(double) * part_cap_);
  }
  int64_t off = 0;
  for (auto& t : ds) {
    t.part = part_buf_ + off;
    off += (int64_t)((t.M + TSK_MT - 1) / TSK_MT) * t.ksplit * TSK_MT * 32;
  }
  Op op{OK_TSK, TP_F64, DT_F64, 0, (int)ds.size(), (int)blocks, push_bytes(ds.data(), ds.size() * sizeof(TskDesc)),
        algorithmic ? fl : 0.0};
  op.bytes = by;
  if (algorithmic) flops_ += fl;
  ops_.push_back(op);
}

void Rec::tc(int prec, int out_dt, std::vector<TcDesc> ds, bool algorithmic) {
  if (ds.empty()) return;
  if (prec == TP_F64 && out_dt == DT_F64 && scratch_ && !ctx_->tuning) {
    std::vector<TskDesc> ts;
    std::vector<TcDesc> rest;
    for (const auto& d : ds) {
      TskDesc t;
      if (tsk_from(d, t)) ts.push_back(t);
      else rest.push_back(d);
    }
    if (!ts.empty()) {
      tsk(std::move(ts), algorithmic);
      ds.swap(rest);
      if (ds.empty()) return;
    }
  }
  // the descriptors of one group are independent, so families (and the
  // skinny-kernel members of a family) may run as separate launches
  std::vector<TcDesc> fam[N_FAMILIES];
  {
    const int f0 = tile_family(ds[0]);
    bool one = true;
    for (size_t i = 1; i < ds.size() && one; ++i) one = tile_family(ds[i]) == f0;
    if (one) fam[f0].swap(ds);
    else
      for (const auto& d : ds) fam[tile_family(d)].push_back(d);
  }
  for (int f = 0; f < N_FAMILIES; ++f) {
    if (fam[f].empty()) continue;
    std::vector<TcDesc> sk, rest;
    size_t nsk = 0;
    for (const auto& d : fam[f]) nsk += (f != 2 && skinny_fits(d)) ? 1 : 0;
    if (nsk == 0) rest.swap(fam[f]);
    else if (nsk == fam[f].size()) sk.swap(fam[f]);
    else
      for (const auto& d : fam[f]) ((f != 2 && skinny_fits(d)) ? sk : rest).push_back(d);
    const uint64_t key[2] = {sk.empty() ? 0 : tune_key(prec, out_dt, f, true, sk),
                             rest.empty() ? 0 : tune_key(prec, out_dt, f, false, rest)};
    bool tuned = ctx_->tuning && scratch_ && !plain_;
    for (int part = 0; part < 2; ++part)
      if (key[part] && ctx_->tuned.count(key[part])) tuned = true;
    if (!tuned) {
      // heuristic: the skinny members in one skinny launch when they fill the
      // chip, everything else in one tiled launch
      // (a declined skinny launch leaves the descriptors as they were; all
      // of them then go to the tiled launch, in their original order)
      std::vector<TcDesc>* tiled;
      if (!sk.empty() && tcs_launch(prec, out_dt, sk, algorithmic)) tiled = &rest;
      else if (sk.empty()) tiled = &rest;
      else if (rest.empty()) tiled = &sk;
      else tiled = &fam[f];
      if (tiled->empty()) continue;
      const int tile = pick_tile(f, *tiled);
      tc_launch(prec, out_dt, tile, std::move(*tiled), algorithmic, true);
      continue;
    }
    for (int part = 0; part < 2; ++part) {
      std::vector<TcDesc>& X = part == 0 ? sk : rest;
      if (X.empty()) continue;
      int choice = HEURISTIC;
      auto it = ctx_->tuned.find(key[part]);
      if (it != ctx_->tuned.end()) {
        choice = it->second;
      } else if (ctx_->tuning && scratch_ && !plain_) {
        bool idempotent = true;
        for (const auto& d : X) idempotent = idempotent && d.beta == 0.0;
        if (idempotent) choice = tune(prec, out_dt, f, part == 0, X, key[part]);
      }
      apply_choice(prec, out_dt, f, choice, X, algorithmic);
    }
  }
}

void Rec::apply_choice(int prec, int out_dt, int fam, int choice, std::vector<TcDesc> ds, bool algorithmic) {
  if (choice == HEURISTIC || choice == SKINNY) {
    bool fits = true;
    for (const auto& d : ds) fits = fits && fam != 2 && skinny_fits(d);
    if (fits && tcs_launch(prec, out_dt, ds, algorithmic)) return;
    const int tile = pick_tile(fam, ds);
    tc_launch(prec, out_dt, tile, std::move(ds), algorithmic, true);
    return;
  }
  const bool split = choice < NO_SPLIT;
  tc_launch(prec, out_dt, split ? choice : choice - NO_SPLIT, std::move(ds), algorithmic, split);
}

// Times every launch shape of the group on its real operands (the group is
// idempotent: beta = 0), keeps the fastest for the signature.  Work recorded
// before is flushed first; each candidate runs twice and its second run is
// timed.
int Rec::tune(int prec, int out_dt, int fam, bool skinny, const std::vector<TcDesc>& ds, uint64_t key) {
  std::vector<int> cand;
  if (skinny) cand.push_back(SKINNY);
  static const std::vector<int> TILES[N_FAMILIES] = {
      {TT_256x16, TT_64x16, TT_128x32, TT_64x32}, {TT_128x32, TT_64x32, TT_64x64}, {TT_32x128, TT_64x32},
      {TT_128x48, TT_64x32, TT_64x64},           {TT_64x80, TT_64x64, TT_64x32},  {TT_64x64, TT_64x32, TT_128x32}};
  for (int t : TILES[fam]) {
    cand.push_back(t);
    cand.push_back(NO_SPLIT + t);
  }
  flush(*scratch_);
  int best = HEURISTIC;
  float best_ms = 0.f;
  for (int c : cand) {
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {
      void* e0 = dev::event_create();
      void* e1 = dev::event_create();
      dev::event_record(e0, ctx_->stream);
      apply_choice(prec, out_dt, fam, c, ds, false);
      flush(*scratch_);
      dev::event_record(e1, ctx_->stream);
      dev::sync(ctx_->stream);
      ms = dev::event_ms(e0, e1);
      dev::event_destroy(e0);
      dev::event_destroy(e1);
    }
    if (best == HEURISTIC || ms < best_ms) {
      best = c;
      best_ms = ms;
    }
  }
  ctx_->tuned[key] = best;
  return best;
}

// The skinny kernel takes a group of fitting contractions whose B tiles
// stage in 64 KB of shared memory and that give at least one 64-row group
// per CU.  Returns false (nothing recorded) when the group does not qualify.

bool Rec::tcs_launch(int prec, int out_dt, std::vector<TcDesc>& ds, bool algorithmic) {
  int maxN = 0, maxK = 0;
  int64_t groups = 0;
  for (const auto& d : ds) {
    if (!skinny_fits(d)) return false;
    maxN = std::max(maxN, d.N);
    maxK = std::max(maxK, d.K);
    groups += (d.M + 63) / 64;
  }
  const int kq = prec == TP_BF16 ? 32 : 4;   // k per MFMA step
  const int nb = (maxN + 15) / 16, kp = (maxK + kq - 1) / kq * kq;
  if (groups < 256 || groups >= INT_MAX || tcs_lds_bytes(prec, nb, kp) > 64 * 1024) return false;
  int64_t base = 0;
  double fl = 0.0;
  for (auto& d : ds) {
    d.tile_base = (int32_t)base;
    d.tiles_n = 1;
    d.ksplit = 1;
    d.kslice = d.K;
    d.part = nullptr;
    base += (d.M + 63) / 64;
    fl += 2.0 * d.M * (double)d.N * d.K;
  }
  Op op{OK_TCS, prec, out_dt, TT_S16 + nb - 1, (int)ds.size(), (int)groups,
        push_bytes(ds.data(), ds.size() * sizeof(TcDesc)), algorithmic ? fl : 0.0};
  for (const auto& d : ds) op.bytes += tc_bytes(prec, out_dt, d);
  op.ksm = prec == TP_BF16 ? (kp <= 64 ? 2 : 4) : (kp <= 32 ? 8 : 16);
  op.kp = kp;
  if (algorithmic) flops_ += fl;
  ops_.push_back(op);
  return true;
}

void Rec::tc_launch(int prec, int out_dt, int tile, std::vector<TcDesc> ds, bool algorithmic, bool allow_split) {
  const int mt = tile_mt(tile), nt = tile_nt(tile);
  const int kt = prec == TP_BF16 ? 32 : 16;
  // Split K when the output tiles leave most CUs idle and K is long: each
  // slice keeps at least two chunks of K, and a second launch sums the
  // slices in order (no cross-workgroup synchronisation inside the kernel).
  int64_t plain = 0, maxK = 0;
  for (const auto& d : ds) {
    plain += (int64_t)((d.M + mt - 1) / mt) * ((d.N + nt - 1) / nt);
    maxK = std::max<int64_t>(maxK, d.K);
  }
  int ksplit = 1;
  if (allow_split && scratch_ && plain < 128 && maxK >= 8 * kt) {
    ksplit = (int)std::min<int64_t>({32, (512 + plain - 1) / plain, maxK / (2 * kt)});
    if (ksplit < 2) ksplit = 1;
  }
  // the partial buffer is reused by every split launch of this recorder:
  // launches run in stream order and each reduction finishes its slices
  // before the next contraction starts
  double* part = nullptr;
  if (ksplit > 1) {
    const size_t need = (size_t)plain * ksplit * mt * nt;
    if (need > part_cap_) {
      part_cap_ = std::max(need, part_cap_ * 2);
      part_buf_ = (double*)scratch_->alloc(sizeof(double) * part_cap_);
    }
    part = part_buf_;
  }
  int64_t tiles = 0, tbase = 0;
  double fl = 0.0;
  for (auto& d : ds) {
    d.tiles_n = (d.N + nt - 1) / nt;
    const int64_t dt = (int64_t)((d.M + mt - 1) / mt) * d.tiles_n;
    d.ksplit = ksplit;
    d.kslice = ksplit > 1 ? (int)(((d.K + ksplit - 1) / ksplit + kt - 1) / kt * kt) : d.K;
    d.part = part ? part + tbase * ksplit * mt * nt : nullptr;
    d.tile_base = (int32_t)tiles;
    tiles += dt * ksplit;
    tbase += dt;
    fl += 2.0 * d.M * (double)d.N * d.K;
  }
  PE_REQUIRE(tiles < INT_MAX, "too many tiles in one launch");
  Op op{OK_TC, prec, out_dt, tile, (int)ds.size(), (int)tiles, push_bytes(ds.data(), ds.size() * sizeof(TcDesc)),
        algorithmic ? fl : 0.0};
  for (const auto& d : ds) op.bytes += tc_bytes(prec, out_dt, d);
  if (algorithmic) flops_ += fl;
  ops_.push_back(op);
  if (ksplit > 1) ops_.push_back(Op{OK_TCR, prec, out_dt, tile, (int)ds.size(), (int)tbase, op.off, 0.0});
}

void Rec::kb(int prec, int out_dt, std::vector<KbDesc> ds, bool algorithmic) {
  if (ds.empty()) return;
  int nb1 = 1, lup = 4, pqp = 4, qmax = 1;
  int64_t blocks = 0;
  double fl = 0.0, by = 0.0;
  const double es = prec == TP_F64 ? 8.0 : 4.0, os = out_dt == DT_F64 ? 8.0 : 4.0;
  for (auto& d : ds) {
    PE_REQUIRE(kb_fits(d, prec), "fused contraction outside the kernel's limits");
    nb1 = std::max(nb1, d.dr.size * d.p.size > 16 ? 2 : 1);
    lup = std::max(lup, (d.lu.size + 3) / 4 * 4);
    pqp = std::max(pqp, (d.p.size * d.q.size + 3) / 4 * 4);
    qmax = std::max(qmax, d.q.size);
    d.tile_base = (int32_t)blocks;
    blocks += (d.r.size + 15) / 16;
    fl += kb_flops(d);
    by += es * ((double)d.r.size * d.lu.size * d.q.size + (double)d.lu.size * d.dr.size * d.p.size +
                (double)d.p.size * d.q.size * d.gs.size) +
          os * (double)d.r.size * d.dr.size * d.gs.size;
  }
  PE_REQUIRE(blocks < INT_MAX && kb_lds_bytes(prec, nb1, lup, pqp, qmax) <= 64 * 1024, "fused contraction too large");
  Op op{OK_KB, prec, out_dt, TT_KB16 + nb1 - 1, (int)ds.size(), (int)blocks,
        push_bytes(ds.data(), ds.size() * sizeof(KbDesc)), algorithmic ? fl : 0.0};
  op.ksm = lup;
  op.kp = pqp;
  op.q = qmax;
  op.bytes = by;
  if (algorithmic) flops_ += fl;
  ops_.push_back(op);
}

void Rec::k2(std::vector<K2Desc> ds, double flops) {
  if (ds.empty()) return;
  int64_t units = 0;
  double by = 0.0;
  int chmax = 1, xmin = INT_MAX;
  for (auto& d : ds) {
    chmax = std::max(chmax, std::max(d.A, d.Y));
    PE_REQUIRE(d.X >= 1 && d.A >= 1 && d.E >= 1 && d.Y >= 1 && d.X <= K2_CHI && d.A <= K2_CHI && d.E <= K2_CHI &&
                   d.Y <= K2_CHI,
               "two-row column step: bond outside the fused kernel's range");
    units += d.E;
    xmin = std::min(xmin, d.X);
    // algorithmic bytes: the incoming environment, both boundary tensors, four sites, the outgoing environment
    by += 8.0 * ((double)d.X * 256 * d.A + (double)d.A * 16 * d.E + (double)d.X * 16 * d.Y + 4 * 512.0 +
                 (double)d.Y * 256 * d.E);
  }
  // x slices.  One workgroup per output value fills the chip's compute
  // units (one workgroup each) in rounds; when the last round would run
  // mostly empty, each value's x range is cut into ns slices.  Model, in
  // units of one value's full x loop: rounds * (1/ns + eps) for the slices
  // plus 2 eps ns for the last slice's sum over the partials, eps the cost
  // of one partial result's trip through memory and of a slice's set-up
  // (0.03 fits the measured column steps of the 8x8 D=4 chi=32 lattice:
  // three slices, 387 us against 412 us with six and 518 us with one).
  constexpr int CUS = 256;
  constexpr double EPS = 0.03;
  int ns = 1;
  if (scratch_ && units < 8 * CUS) {
    double best = std::ceil((double)units / CUS);
    for (int s = 2; s <= 8 && 2 * s <= xmin; ++s) {
      const double c = std::ceil((double)units * s / CUS) * (1.0 / s + EPS) + 2.0 * EPS * s;
      if (c < best - 1e-9) {
        best = c;
        ns = s;
      }
    }
  }
  int64_t blocks = 0, parts = 0;
  for (auto& d : ds) {
    d.ns = ns;
    d.block_base = (int32_t)blocks;
    blocks += (int64_t)d.E * ns;
    d.cnt_base = cq_slots_;
    d.part = nullptr;
    if (ns > 1) {
      cq_slots_ += d.E;
      parts += (int64_t)d.E * ns * K2_PART;
    }
  }
  PE_REQUIRE(blocks < INT_MAX / 8, "fused two-row step too large");
  if (parts > 0) {
    // shared with the other split launches of this recorder (stream order)
    if ((size_t)parts > part_cap_) {
      part_cap_ = std::max((size_t)parts, part_cap_ * 2);
      part_buf_ = (double*)scratch_->alloc(sizeof(double) * part_cap_);
    }
    int64_t off = 0;
    for (auto& d : ds) {
      d.part = part_buf_ + off;
      off += (int64_t)d.E * ns * K2_PART;
    }
  }
  Op op{OK_K2, TP_F64, DT_F64, TT_K2, (int)ds.size(), (int)blocks, push_bytes(ds.data(), ds.size() * sizeof(K2Desc)),
        flops};
  op.bytes = by;
  op.kp = chmax;
  flops_ += flops;
  ops_.push_back(op);
}

void Rec::kc(std::vector<KcDesc> ds, double flops) {
  if (ds.empty()) return;
  // A workgroup stages both sites and one top boundary slab for KC_W waves'
  // worth of work; in a launch of many workgroups (batches) it makes xr
  // passes over consecutive x groups so that the staging is shared, while
  // keeping at least 1024 workgroups (four per compute unit) in flight.
  int64_t one = 0;
  for (const auto& d : ds) one += (int64_t)((d.X + KC_W - 1) / KC_W) * d.Ne;
  const int xr = (int)std::max<int64_t>(1, std::min<int64_t>(4, one / 1024));
  int64_t blocks = 0;
  for (auto& d : ds) {
    PE_REQUIRE(d.X >= 1 && d.A >= 1 && d.Ne >= 1 && d.A <= K2_CHI, "one-row chain step: bond outside the fused kernel's range");
    d.block_base = (int32_t)blocks;
    d.xr = xr;
    const int64_t groups = (d.X + KC_W - 1) / KC_W;
    blocks += (groups + xr - 1) / xr * d.Ne;
  }
  PE_REQUIRE(blocks < INT_MAX / 8, "one-row chain step too large");
  flops_ += flops;
  ops_.push_back(Op{OK_KC, TP_F64, DT_F64, 0, (int)ds.size(), (int)blocks, push_bytes(ds.data(), ds.size() * sizeof(KcDesc)),
                    flops});
}

// Householder QR of every block of the group.  Blocks that fit a
// register-resident variant run as one grouped launch; taller blocks with at
// most TSQR_NMAX columns are factored as a tree (TSQR): row blocks of at most
// TSQR_LEAF rows in parallel, then the stack of their R factors recursively,
// and Q rebuilt by one grouped contraction per level.  Every node keeps
// R_ii >= 0, so Q and R are the unique factors with that sign convention,
// the ones a single Householder QR gives.  Wider blocks use the streaming
// kernel.
void Rec::qr(const std::vector<QrDesc>& ds) {
  if (ds.empty()) return;
  int mm = 0, nn = 0;
  for (const auto& d : ds) {
    PE_REQUIRE(d.m >= d.n && d.n >= 1 && d.n <= 1024, "QR shape");
    mm = std::max(mm, d.m);
    nn = std::max(nn, d.n);
  }
  const int variant = qr_variant_for(mm, nn);
  if (variant == QR_CQ) {
    if (qr_depth_ == 0) qr_used_ = 0;   // earlier QR ops are ordered before this one on the stream
    qr_cq(ds, nn <= 16 ? 1 : 2);
    return;
  }
  if (variant < 0 && nn <= TSQR_NMAX) {
    if (qr_depth_ == 0) qr_used_ = 0;   // earlier QR ops are ordered before this one on the stream
    ++qr_depth_;
    qr_tall(ds);
    --qr_depth_;
    return;
  }
  ops_.push_back(Op{OK_QR, 0, 0, variant, (int)ds.size(), (int)ds.size(),
                    push_bytes(ds.data(), ds.size() * sizeof(QrDesc)), 0.0});
}

// CholeskyQR2 over several workgroups per block: each block gets its own
// workspace region and arrival counter; a launch holds at most CQ_MAXWG
// workgroups, so that all of them are resident together.
void Rec::qr_cq(const std::vector<QrDesc>& ds, int nb) {
  size_t i = 0;
  while (i < ds.size()) {
    std::vector<CqDesc> cs;
    int blocks = 0;
    for (; i < ds.size(); ++i) {
      const int P = (ds[i].m + CQ_ROWS - 1) / CQ_ROWS;
      PE_REQUIRE(P <= CQ_MAXP, "CholeskyQR2 block too tall");
      if (blocks + P > CQ_MAXWG) break;
      CqDesc c{};
      c.q = ds[i];
      c.q.W = nullptr;
      c.ws = qr_scratch(cq_ws_doubles(ds[i].m, 16 * nb));   // offsets follow the launch's column blocks
      c.cnt = cq_slots_++;
      c.P = P;
      c.block_base = blocks;
      blocks += P;
      cs.push_back(c);
    }
    ops_.push_back(Op{OK_CQ, 0, 0, nb, (int)cs.size(), blocks, push_bytes(cs.data(), cs.size() * sizeof(CqDesc)), 0.0});
  }
}

double* Rec::qr_scratch(size_t n) {
  PE_REQUIRE(scratch_ != nullptr, "tall QR needs a scratch arena");
  n = (n + 31) & ~(size_t)31;   // 256-byte granules
  if (qr_used_ + n > qr_cap_) {
    // regions carved earlier in this QR stay valid: the old buffer lives in the arena
    qr_cap_ = std::max(2 * qr_cap_, n + (size_t(1) << 20));
    qr_buf_ = (double*)scratch_->alloc(sizeof(double) * qr_cap_);
    qr_used_ = 0;
  }
  double* p = qr_buf_ + qr_used_;
  qr_used_ += n;
  return p;
}

void Rec::qr_tall(const std::vector<QrDesc>& ds) {
  std::vector<QrDesc> leaves, stacks;
  std::vector<TcDesc> rebuild;
  for (const QrDesc& d : ds) {
    const int m = d.m, n = d.n;
    const int b = (m + TSQR_LEAF - 1) / TSQR_LEAF;   // row blocks, each of >= TSQR_LEAF/2 >= n rows
    double* Qb = qr_scratch((size_t)m * n);          // Q of every row block, row-major
    double* S = qr_scratch((size_t)b * n * n);       // stacked R factors
    double* QS = qr_scratch((size_t)b * n * n);      // Q of the stack
    int row0 = 0;
    for (int i = 0; i < b; ++i) {
      const int r = m / b + (i < m % b ? 1 : 0);
      PE_REQUIRE(r >= n, "TSQR block shorter than its width");
      leaves.push_back(QrDesc{d.A + row0 * d.sAr, d.sAr, d.sAc, Qb + (int64_t)row0 * n, n, 1,
                              S + (int64_t)i * n * n, n, 1, nullptr, r, n});
      // final rows of block i: Q[row0 .. row0+r) = Qb_i . QS[i*n .. (i+1)*n)
      TV C;
      C.p = d.Q + row0 * d.sQr;
      C.dt = DT_F64;
      C.idx = "ik";
      C.dim = {r, n};
      C.str = {d.sQr, d.sQc};
      rebuild.push_back(tc_build(C, dense(Qb + (int64_t)row0 * n, DT_F64, "ij", {r, n}),
                                 dense(QS + (int64_t)i * n * n, DT_F64, "jk", {n, n})));
      row0 += r;
    }
    stacks.push_back(QrDesc{S, n, 1, QS, n, 1, d.R, d.sRr, d.sRc, nullptr, b * n, n});
  }
  for (const QrDesc& l : leaves) PE_REQUIRE(qr_variant_for(l.m, l.n) >= 0, "TSQR leaf without a register variant");
  qr(leaves);
  qr(stacks);   // recursion while the stack is still taller than a register block
  tc(TP_F64, DT_F64, rebuild, false);   // (grouped with the same rules as every contraction)
}

void Rec::reduce(std::vector<RedDesc> ds) {
  if (ds.empty()) return;
  int blocks = 0;
  for (auto& d : ds) {
    d.nblocks = (int)std::max<int64_t>(1, std::min<int64_t>(256, (d.n + 8191) / 8192));
    d.block_base = blocks;
    d.part_base = partials_ + blocks;
    blocks += d.nblocks;
  }
  partials_ += blocks;
  ops_.push_back(Op{OK_RED, 0, 0, 0, (int)ds.size(), blocks, push_bytes(ds.data(), ds.size() * sizeof(RedDesc)), 0.0});
}

void Rec::ew(std::vector<EwDesc> ds) {
  if (ds.empty()) return;
  int blocks = 0;
  for (auto& d : ds) {
    d.nblocks = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (d.n + 1023) / 1024));
    d.block_base = blocks;
    blocks += d.nblocks;
  }
  ops_.push_back(Op{OK_EW, 0, 0, 0, (int)ds.size(), blocks, push_bytes(ds.data(), ds.size() * sizeof(EwDesc)), 0.0});
}

void Rec::sep(const std::vector<SepDesc>& ds) {
  if (ds.empty()) return;
  int dmax = 1;
  for (const auto& d : ds) dmax = std::max(dmax, (int)d.dmax);
  Op op{OK_SEP, 0, 0, 0, (int)ds.size(), (int)ds.size(), push_bytes(ds.data(), ds.size() * sizeof(SepDesc)), 0.0};
  op.kp = dmax;
  ops_.push_back(op);
}

void* Rec::aux(Arena& arena, const void* data, size_t bytes) {
  void* d = arena.alloc(bytes);
  aux_.push_back({d, {push_bytes(data, bytes), bytes}});
  return d;
}

void Rec::issue(const uint8_t* dblob, double* partials, unsigned* counters, bool timed, hipStream_t s) {
  for (auto& a : aux_) dev::d2d(a.first, dblob + a.second.first, a.second.second, s);
  launch_cq_clear(counters, cq_slots_, s);
  for (size_t i = 0; i < ops_.size(); ++i) {
    const Op& op = ops_[i];
    const void* d = dblob + op.off;
    void* e0 = nullptr;
    if (timed && (op.kind == OK_TC || op.kind == OK_TCS || op.kind == OK_KB || op.kind == OK_K2)) {
      e0 = dev::event_create();
      dev::event_record(e0, s);
    }
    switch (op.kind) {
      case OK_TC: launch_tc(op.prec, op.out_dt, op.tile, (const TcDesc*)d, op.nd, op.grid, s); break;
      case OK_TCR: launch_tc_reduce(op.out_dt, op.tile, (const TcDesc*)d, op.nd, op.grid, s); break;
      case OK_TCS:
        launch_tcs(op.prec, op.out_dt, op.tile - TT_S16 + 1, op.ksm, (const TcDesc*)d, op.nd, op.grid, op.kp, s);
        break;
      case OK_K2: launch_k2((const K2Desc*)d, op.nd, op.grid, op.kp, counters, s); break;
      case OK_KC: launch_kc((const KcDesc*)d, op.nd, op.grid, s); break;
      case OK_TSK: launch_tsk((const TskDesc*)d, op.nd, op.grid, counters, s); break;
      case OK_KB:
        launch_kb(op.prec, op.out_dt, op.tile - TT_KB16 + 1, (const KbDesc*)d, op.nd, op.grid, op.ksm, op.kp, op.q, s);
        break;
      case OK_QR:
        if (op.tile >= 0) launch_qr_reg(op.tile, (const QrDesc*)d, op.nd, s);
        else launch_qr((const QrDesc*)d, op.nd, s);
        break;
      case OK_CQ: launch_cq(op.tile, (const CqDesc*)d, op.nd, op.grid, counters, s); break;
      case OK_RED: launch_reduce((const RedDesc*)d, op.nd, op.grid, partials, s); break;
      case OK_EW: launch_ew((const EwDesc*)d, op.nd, op.grid, s); break;
      case OK_SEP: launch_sep((const SepDesc*)d, op.nd, op.kp, s); break;
    }
    if (e0) {
      void* e1 = dev::event_create();
      dev::event_record(e1, s);
      events_.push_back(Timed{e0, e1, tc_stat_index(op.prec, op.out_dt, op.tile), op.flops, op.bytes});
    }
  }
}

void Rec::flush(Arena& arena) {
  if (ops_.empty()) return;
  if (plain_) {
    hipStream_t s = ctx_->stream;
    uint8_t* dblob = (uint8_t*)arena.alloc(blob_.size());
    double* partials = (double*)arena.alloc(sizeof(double) * (size_t)std::max(partials_, 1));
    unsigned* counters = (unsigned*)arena.alloc(sizeof(unsigned) * (size_t)std::max(cq_slots_, 1));
    dev::h2d(dblob, blob_.data(), blob_.size(), s);
    issue(dblob, partials, counters, false, s);
    dev::sync(s);   // the host copy of the descriptors is reused by the next recording
  } else if (ctx_->graphs && !ctx_->profile && !ctx_->tuning) {
    flush_graph();
  } else {
    hipStream_t s = ctx_->stream;
    uint8_t* dblob = (uint8_t*)arena.alloc(blob_.size());
    double* partials = (double*)arena.alloc(sizeof(double) * (size_t)std::max(partials_, 1));
    unsigned* counters = (unsigned*)arena.alloc(sizeof(unsigned) * (size_t)std::max(cq_slots_, 1));
    void* host = ctx_->pinned_get(blob_.size());
    pinned_.push_back({host, blob_.size()});
    std::memcpy(host, blob_.data(), blob_.size());
    dev::h2d(dblob, host, blob_.size(), s);
    issue(dblob, partials, counters, ctx_->profile, s);
  }
  ops_.clear();
  blob_.clear();
  aux_.clear();
  partials_ = 0;
  cq_slots_ = 0;
}

// Graph replay: the launch sequence is identified by everything its kernels
// and copies read from the host side (descriptor bytes with their device
// pointers, launch shapes, copy destinations).  A byte-identical sequence
// replays the instantiated graph with the descriptors it captured; the first
// occurrence uploads a descriptor copy owned by the cache and is captured.
void Rec::flush_graph() {
  hipStream_t s = ctx_->stream;
  std::vector<uint8_t> key = blob_;
  auto put = [&key](const void* p, size_t n) {
    const uint8_t* b = (const uint8_t*)p;
    key.insert(key.end(), b, b + n);
  };
  for (const Op& op : ops_) {
    const int32_t f[10] = {op.kind, op.prec, op.out_dt, op.tile, op.nd, op.grid, (int32_t)op.off, op.ksm, op.kp, op.q};
    put(f, sizeof(f));
  }
  for (const auto& a : aux_) {
    put(&a.first, sizeof(a.first));
    put(&a.second, sizeof(a.second));
  }
  put(&partials_, sizeof(partials_));
  put(&cq_slots_, sizeof(cq_slots_));
  uint64_t h = 1469598103934665603ull;   // FNV-1a
  for (uint8_t c : key) h = (h ^ c) * 1099511628211ull;
  auto& bucket = ctx_->graph_cache[h];
  for (const Ctx::Graph& g : bucket)
    if (g.key == key) {
      dev::graph_launch(g.exec, s);
      return;
    }
  if (ctx_->graph_count >= Ctx::GRAPH_MAX) {
    dev::sync(s);   // no cached graph is still executing
    ctx_->clear_graphs();
  }
  Ctx::Graph g;
  g.dblob = (uint8_t*)ctx_->pool.alloc(blob_.size());
  g.partials = (double*)ctx_->pool.alloc(sizeof(double) * (size_t)std::max(partials_, 1));
  g.counters = (unsigned*)ctx_->pool.alloc(sizeof(unsigned) * (size_t)std::max(cq_slots_, 1));
  void* host = ctx_->pinned_get(blob_.size());
  pinned_.push_back({host, blob_.size()});
  std::memcpy(host, blob_.data(), blob_.size());
  dev::h2d(g.dblob, host, blob_.size(), s);
  // recording executes nothing, so it needs no ordering with the caller's
  // stream; the graph is then launched there
  if (!ctx_->capture_stream) ctx_->capture_stream = dev::stream_create();
  hipStream_t cs = ctx_->capture_stream;
  dev::capture_begin(cs);
  try {
    issue(g.dblob, g.partials, g.counters, false, cs);
    g.exec = dev::capture_end(cs);
  } catch (...) {
    dev::capture_abort(cs);
    ctx_->pool.release(g.dblob);
    ctx_->pool.release(g.partials);
    ctx_->pool.release(g.counters);
    throw;
  }
  dev::graph_launch(g.exec, s);
  g.key.swap(key);
  ctx_->graph_cache[h].push_back(std::move(g));
  ++ctx_->graph_count;
}

void Rec::run(Arena& arena) {
  flush(arena);
  // staging buffers and descriptors stay valid until the stream drains
  dev::sync(ctx_->stream);
  for (auto& e : events_) {
    ctx_->st_ms[e.key] += dev::event_ms(e.e0, e.e1);
    ctx_->st_flops[e.key] += e.flops;
    ctx_->st_bytes[e.key] += e.bytes;
    ctx_->st_launch[e.key] += 1;
    dev::event_destroy(e.e0);
    dev::event_destroy(e.e1);
  }
  events_.clear();
  for (auto& p : pinned_) ctx_->pinned_put(p.first, p.second);
  pinned_.clear();
}

Rec::Rec(Ctx* c, Arena* scratch) : ctx_(c), scratch_(scratch) {
  blob_.swap(ctx_->blob_spare);   // its capacity, not its contents
  blob_.clear();
}

Rec::~Rec() {
  blob_.clear();
  if (blob_.capacity() > ctx_->blob_spare.capacity()) ctx_->blob_spare.swap(blob_);
  if (!pinned_.empty() || !events_.empty()) {
    try {
      dev::sync(ctx_->stream);
    } catch (...) {
    }
    for (auto& e : events_) {
      dev::event_destroy(e.e0);
      dev::event_destroy(e.e1);
    }
    for (auto& p : pinned_) ctx_->pinned_put(p.first, p.second);
  }
}

}  // namespace pe
