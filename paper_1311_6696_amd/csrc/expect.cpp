// Local expectation values from the sandwich (arXiv:1311.6696, Sec. 2):
// each row is contracted between the top boundary above it and the bottom
// boundary below it, giving <psi|psi>, <S^z> and horizontal bond energies;
// vertical bonds come from the two-row sandwich between T_{r-1} and B_{r+2}.
// Operators act on the ket layer; every ratio takes numerator and
// denominator from the same sandwich.
//
// All rows of all environments run together: the left and right column
// environments of every row advance in lockstep (one grouped launch per
// stage), then all operator insertions of all rows form two more batched
// levels, then every scalar is one reduction.
#include <array>
#include <map>

#include "chains.hpp"

namespace pe {
namespace {

// groups of consecutive items whose scratch fits the budget (at least one each)
std::vector<std::pair<size_t, size_t>> budget_groups(const std::vector<size_t>& sz, size_t budget) {
  std::vector<std::pair<size_t, size_t>> g;
  size_t i = 0;
  for (size_t k = 0; k < sz.size(); ++k)
    if (sz[k] > budget)
      throw Error(ST_OOM, "one sandwich needs " + std::to_string(sz[k]) + " bytes of workspace, above the cap of " +
                              std::to_string(budget) + " (peps_ctx_set_workspace)");
  while (i < sz.size()) {
    size_t j = i, tot = 0;
    while (j < sz.size() && (j == i || tot + sz[j] <= budget)) tot += sz[j++];
    g.push_back({i, j});
    i = j;
  }
  return g;
}

// One-row sandwich of row r (between T_{r-1} and B_{r+1}).
struct RJob {
  peps_env* e;
  peps_env* owner;   // receives the results: e itself, or the lattice e is the transpose of
  bool tr;           // row r of a transposed lattice: only its bonds (vertical bonds of column r)
  int r, Lc;
  const Mps* T;
  const Mps* B;
  std::vector<const Site*> s;
  std::vector<int64_t> bT, bB, Dl;
  std::vector<void*> L, R;
  double* nuL;   // Lc+1 squared norms of the raw left steps
  double* nuR;
  double* dots;  // D[0..Lc], sz nums [Lc], bond nums [3*(Lc-1)]
};

// Runs what `rec` holds and reads each job's Lc+1 overlaps and left/right
// squared step norms back in one transfer.
void run_and_read_dots(Rec& rec, Arena& call, const std::vector<RJob>& rj, hipStream_t s,
                       std::vector<std::vector<double>>& hd, std::vector<std::vector<double>>& hl,
                       std::vector<std::vector<double>>& hr) {
  Gather g;
  std::vector<std::array<size_t, 3>> off(rj.size());
  for (size_t k = 0; k < rj.size(); ++k) {
    const size_t n = (size_t)rj[k].Lc + 1;
    off[k] = {g.add(rj[k].dots, n), g.add(rj[k].nuL, n), g.add(rj[k].nuR, n)};
  }
  g.record(rec, call);
  rec.run(call);
  g.read(s);
  hd.resize(rj.size());
  hl.resize(rj.size());
  hr.resize(rj.size());
  for (size_t k = 0; k < rj.size(); ++k) {
    const size_t n = (size_t)rj[k].Lc + 1;
    hd[k] = g.slice(off[k][0], n);
    hl[k] = g.slice(off[k][1], n);
    hr[k] = g.slice(off[k][2], n);
  }
}

struct R2Job {
  peps_env* e;
  int r, Lc;
  const Mps* T;
  const Mps* B;
  std::vector<const Site*> s1, s2;
  std::vector<int64_t> bT, bB, Dl1, Dl2;
  std::vector<void*> L, R;
  double* nuL;
  double* nuR;
  double* dots;  // D[0..Lc], nums [3*Lc]
};

int64_t env_elems(const RJob& j, int c) { return j.bB[c] * j.Dl[c] * j.Dl[c] * j.bT[c]; }
int64_t env2_elems(const R2Job& j, int c) {
  return j.bB[c] * j.Dl2[c] * j.Dl2[c] * j.Dl1[c] * j.Dl1[c] * j.bT[c];
}

TV envv(const RJob& j, const void* p, int c, const char* lbl, int cdt) {
  return dense(p, cdt, lbl, {j.bB[c], j.Dl[c], j.Dl[c], j.bT[c]});
}
TV env2v(const R2Job& j, const void* p, int c, const char* lbl, int cdt) {
  return dense(p, cdt, lbl, {j.bB[c], j.Dl2[c], j.Dl2[c], j.Dl1[c], j.Dl1[c], j.bT[c]});
}

// scratch (elements) of one row step at column c: P and Q
std::pair<int64_t, int64_t> step_scratch(const RJob& j, int c) {
  const Site& s = *j.s[c];
  const int64_t X = std::max(j.bB[c], j.bB[c + 1]), A = std::max(j.bT[c], j.bT[c + 1]);
  const int64_t Dh = std::max(s.Dl, s.Dr), Dv = std::max(s.Du, s.Dd);
  return {X * Dh * Dh * Dv * Dv * A, X * Dh * Dh * Dv * Dv * A * s.d};
}
std::pair<int64_t, int64_t> step2_scratch(const R2Job& j, int c) {
  const Site& a = *j.s1[c];
  const Site& b = *j.s2[c];
  const int64_t X = std::max(j.bB[c], j.bB[c + 1]), A = std::max(j.bT[c], j.bT[c + 1]);
  const int64_t h1 = std::max(a.Dl, a.Dr), h2 = std::max(b.Dl, b.Dr);
  const int64_t v = std::max(std::max(a.Du, a.Dd), std::max(b.Du, b.Dd));
  const int64_t P = X * h2 * h2 * h1 * h1 * v * v * A;
  return {P, P * std::max(a.d, b.d)};
}

TV step_left(St& st, std::vector<TcDesc>& fin, const RJob& j, int c, const TV& Lin, int op, void* out, void* P,
             void* Q, int cdt) {
  const Site& s = *j.s[c];
  TV T = dense(j.T->tc[c], cdt, "auve", {j.bT[c], j.T->leg[c], j.T->leg[c], j.bT[c + 1]});
  TV y3 = chain_left(st, Lin, T, site_tv(s, op, false, cdt, "plurd"), site_tv(s, 0, false, cdt, "pmvsg"), P, Q, cdt);
  TV B = dense(j.B->tc[c], cdt, "xdgy", {j.bB[c], j.B->leg[c], j.B->leg[c], j.bB[c + 1]});
  TV o = envv(j, out, c + 1, "yrse", cdt);
  fin.push_back(tc_build(o, y3, B));
  st.flops += tc_flops(fin.back());
  return o;
}

TV step_right(St& st, std::vector<TcDesc>& fin, const RJob& j, int c, const TV& Rin, void* out, void* P, void* Q,
              int cdt) {
  const Site& s = *j.s[c];
  TV T = dense(j.T->tc[c], cdt, "auve", {j.bT[c], j.T->leg[c], j.T->leg[c], j.bT[c + 1]});
  TV y3 = chain_right(st, Rin, T, site_tv(s, 0, false, cdt, "plurd"), site_tv(s, 0, false, cdt, "pmvsg"), P, Q, cdt);
  TV B = dense(j.B->tc[c], cdt, "xdgy", {j.bB[c], j.B->leg[c], j.B->leg[c], j.bB[c + 1]});
  TV o = envv(j, out, c, "xlma", cdt);
  fin.push_back(tc_build(o, y3, B));
  st.flops += tc_flops(fin.back());
  return o;
}

TV step2_left(St& st, std::vector<TcDesc>& fin, const R2Job& j, int c, const TV& Lin, int op1, int op2, void* out,
              void* P, void* Q, int cdt) {
  const Site& a = *j.s1[c];
  const Site& b = *j.s2[c];
  TV T = dense(j.T->tc[c], cdt, "auve", {j.bT[c], j.T->leg[c], j.T->leg[c], j.bT[c + 1]});
  TV y3 = chain2_left(st, Lin, T, site_tv(a, op1, false, cdt, "plurd"), site_tv(a, 0, false, cdt, "pmvsg"),
                      site_tv(b, op2, false, cdt, "qLdRD"), site_tv(b, 0, false, cdt, "qMgSG"), P, Q, cdt);
  TV B = dense(j.B->tc[c], cdt, "xDGy", {j.bB[c], j.B->leg[c], j.B->leg[c], j.bB[c + 1]});
  TV o = env2v(j, out, c + 1, "yRSrse", cdt);
  fin.push_back(tc_build(o, y3, B));
  st.flops += tc_flops(fin.back());
  return o;
}

TV step2_right(St& st, std::vector<TcDesc>& fin, const R2Job& j, int c, const TV& Rin, void* out, void* P, void* Q,
               int cdt) {
  const Site& a = *j.s1[c];
  const Site& b = *j.s2[c];
  TV T = dense(j.T->tc[c], cdt, "auve", {j.bT[c], j.T->leg[c], j.T->leg[c], j.bT[c + 1]});
  TV y3 = chain2_right(st, Rin, T, site_tv(a, 0, false, cdt, "plurd"), site_tv(a, 0, false, cdt, "pmvsg"),
                       site_tv(b, 0, false, cdt, "qLdRD"), site_tv(b, 0, false, cdt, "qMgSG"), P, Q, cdt);
  TV B = dense(j.B->tc[c], cdt, "xDGy", {j.bB[c], j.B->leg[c], j.B->leg[c], j.bB[c + 1]});
  TV o = env2v(j, out, c, "xLMlma", cdt);
  fin.push_back(tc_build(o, y3, B));
  st.flops += tc_flops(fin.back());
  return o;
}

// The fused two-row column step (k2_kernel) takes a column whose sites all
// have legs of dimension K2_D and physical dimension 2, float64, bonds up to
// K2_CHI.
bool fuse2(const R2Job& j, int c, int prec) {
  if (prec != TP_F64) return false;
  for (const Site* s : {j.s1[c], j.s2[c]})
    if (s->d != 2 || s->Dl != K2_D || s->Du != K2_D || s->Dr != K2_D || s->Dd != K2_D) return false;
  if (j.T->leg[c] != K2_D || j.B->leg[c] != K2_D) return false;
  for (int64_t b : {j.bT[c], j.bT[c + 1], j.bB[c], j.bB[c + 1]})
    if (b < 1 || b > K2_CHI) return false;
  return true;
}

// Algorithmic flops of one fused column step (those of the unfused chain):
// top boundary, two ket and two bra layers, bottom boundary.
double k2_flops(const K2Desc& d) {
  return 2.0 * d.X * d.E * (256.0 * 16 * d.A + 4 * 131072.0 + 256.0 * 16 * d.Y);
}

// Canonical form of a two-row column step (see K2Desc): the left-to-right
// step as it is, the right-to-left one with incoming and outgoing roles of
// every horizontal leg and bond exchanged.
K2Desc k2_desc(const R2Job& j, int c, bool left, const TV& in, const TV& out, int op1, int op2) {
  const Site& a = *j.s1[c];
  const Site& b = *j.s2[c];
  TV T = dense(j.T->tc[c], DT_F64, "auve", {j.bT[c], j.T->leg[c], j.T->leg[c], j.bT[c + 1]});
  TV B = dense(j.B->tc[c], DT_F64, "xDGy", {j.bB[c], j.B->leg[c], j.B->leg[c], j.bB[c + 1]});
  const TV sv[4] = {site_tv(a, op1, false, DT_F64, "plurd"), site_tv(a, 0, false, DT_F64, "pmvsg"),
                    site_tv(b, op2, false, DT_F64, "qLdRD"), site_tv(b, 0, false, DT_F64, "qMgSG")};
  K2Desc d;
  std::memset(&d, 0, sizeof(d));
  d.L = (const double*)in.p;
  d.T = (const double*)T.p;
  d.B = (const double*)B.p;
  d.O = (double*)const_cast<void*>(out.p);
  for (int k = 0; k < 6; ++k) {
    d.sL[k] = in.str[k];
    d.sO[k] = out.str[k];
  }
  const int h[4] = {3, 1, 2, 0};   // exchange the horizontal roles: (a,u,v,e) -> (e,u,v,a)
  for (int k = 0; k < 4; ++k) {
    d.sT[k] = left ? T.str[k] : T.str[h[k]];
    d.sB[k] = left ? B.str[k] : B.str[h[k]];
  }
  const int hs[5] = {0, 3, 2, 1, 4};   // (p, in, up, out, down) from (p, l, u, r, d)
  for (int v = 0; v < 4; ++v) {
    d.s[v] = (const double*)sv[v].p;
    for (int k = 0; k < 5; ++k) d.ss[v][k] = left ? sv[v].str[k] : sv[v].str[hs[k]];
  }
  d.X = (int32_t)(left ? j.bB[c] : j.bB[c + 1]);
  d.A = (int32_t)(left ? j.bT[c] : j.bT[c + 1]);
  d.E = (int32_t)(left ? j.bT[c + 1] : j.bT[c]);
  d.Y = (int32_t)(left ? j.bB[c + 1] : j.bB[c]);
  return d;
}

// Normalise the raw outputs in place: nu = |X|^2 into `slot`, X /= sqrt(nu).
void normalise(Rec& rec, const std::vector<std::pair<TV, double*>>& outs) {
  std::vector<RedDesc> rd;
  std::vector<EwDesc> ew;
  for (auto& o : outs) {
    const int64_t n = o.first.size();
    rd.push_back(red_desc(o.first.p, nullptr, n, o.second, o.first.dt));
    EwDesc e = ew_desc(EW_RSQRT, o.first.p, o.first.dt, const_cast<void*>(o.first.p), o.first.dt, n);
    e.sptr = o.second;
    ew.push_back(e);
  }
  rec.reduce(std::move(rd));
  rec.ew(std::move(ew));
}

// One single-row sandwich job: row r of e between T_{r-1} and B_{r+1}, its
// environment buffers in `call`; results go to `owner`.
RJob make_row_job(peps_env* e, peps_env* owner, bool tr, int r, Arena& call, size_t esz) {
  const Lattice& L = e->lat;
  const int Lc = L.Lc;
  RJob j;
  j.e = e;
  j.owner = owner;
  j.tr = tr;
  j.r = r;
  j.Lc = Lc;
  j.T = &e->T(r - 1);
  j.B = &e->B(r + 1);
  for (int c = 0; c < Lc; ++c) j.s.push_back(&L.at(r, c));
  for (int c = 0; c <= Lc; ++c) {
    j.bT.push_back(j.T->bond[c]);
    j.bB.push_back(j.B->bond[c]);
    j.Dl.push_back(c < Lc ? L.at(r, c).Dl : L.at(r, Lc - 1).Dr);
  }
  j.L.assign(Lc + 1, nullptr);
  j.R.assign(Lc + 1, nullptr);
  j.L[0] = const_cast<void*>(L.lam[r]);
  j.R[Lc] = const_cast<void*>(L.rho[r]);
  for (int c = 1; c < Lc; ++c) {
    j.L[c] = call.alloc(esz * env_elems(j, c));
    j.R[c] = call.alloc(esz * env_elems(j, c));
  }
  if (Lc >= 1) {
    j.L[Lc] = call.alloc(esz * env_elems(j, Lc));
    j.R[0] = call.alloc(esz * env_elems(j, 0));
  }
  j.nuL = (double*)call.alloc(sizeof(double) * (Lc + 1));
  j.nuR = (double*)call.alloc(sizeof(double) * (Lc + 1));
  j.dots = (double*)call.alloc(sizeof(double) * (Lc + 1 + Lc + 3 * Lc));
  return j;
}

// Left and right column environments of every job (normalised, squared
// norms in nuL/nuR), grouped by the scratch budget; one grouped launch per
// stage and column step.
void column_envs(Rec& rec, Arena& call, Scratch& scr, std::vector<RJob>& rj, std::vector<R2Job>& r2, int prec,
                 int cdt, size_t esz, size_t budget) {
  struct Slot {
    int kind;   // 0 one-row left, 1 one-row right, 2 two-row left, 3 two-row right
    size_t job;
  };
  std::vector<Slot> slots;
  std::vector<size_t> sz;
  for (size_t i = 0; i < rj.size(); ++i)
    for (int k = 0; k < 2; ++k) {
      size_t m = 0;
      for (int c = 0; c < rj[i].Lc; ++c) {
        auto pq = step_scratch(rj[i], c);
        m = std::max(m, (size_t)(pq.first + pq.second));
      }
      slots.push_back({k, i});
      sz.push_back(m * esz);
    }
  for (size_t i = 0; i < r2.size(); ++i)
    for (int k = 2; k < 4; ++k) {
      size_t m = 0;
      for (int c = 0; c < r2[i].Lc; ++c) {
        auto pq = step2_scratch(r2[i], c);
        m = std::max(m, (size_t)(pq.first + pq.second));
      }
      slots.push_back({k, i});
      sz.push_back(m * esz);
    }
  for (auto g : budget_groups(sz, budget)) {
    std::vector<void*> P(g.second - g.first), Q(g.second - g.first);
    int maxLc = 0;
    for (size_t i = g.first; i < g.second; ++i) {
      const Slot& sl = slots[i];
      int64_t p = 0, q = 0;
      const int Lc = sl.kind < 2 ? rj[sl.job].Lc : r2[sl.job].Lc;
      maxLc = std::max(maxLc, Lc);
      for (int c = 0; c < Lc; ++c) {
        auto pq = sl.kind < 2 ? step_scratch(rj[sl.job], c) : step2_scratch(r2[sl.job], c);
        p = std::max(p, pq.first);
        q = std::max(q, pq.second);
      }
      P[i - g.first] = scr.get(esz * p);
      Q[i - g.first] = scr.get(esz * q);
    }
    for (int s = 0; s < maxLc; ++s) {
      St st1(3, prec), st2(5, prec);
      std::vector<TcDesc> fin;
      std::vector<K2Desc> k2s;
      double k2f = 0.0;
      std::vector<std::pair<TV, double*>> outs;
      for (size_t i = g.first; i < g.second; ++i) {
        const Slot& sl = slots[i];
        void* p = P[i - g.first];
        void* q = Q[i - g.first];
        if (sl.kind < 2) {
          RJob& j = rj[sl.job];
          if (s >= j.Lc) continue;
          const double f0 = st1.flops;
          if (sl.kind == 0) {
            const int c = s;
            TV o = step_left(st1, fin, j, c, envv(j, j.L[c], c, "xlma", cdt), 0, j.L[c + 1], p, q, cdt);
            outs.push_back({o, j.nuL + c + 1});
          } else {
            const int c = j.Lc - 1 - s;
            TV o = step_right(st1, fin, j, c, envv(j, j.R[c + 1], c + 1, "yrse", cdt), j.R[c], p, q, cdt);
            outs.push_back({o, j.nuR + c});
          }
          j.e->flops += st1.flops - f0;
        } else {
          R2Job& j = r2[sl.job];
          if (s >= j.Lc) continue;
          const double f0 = st2.flops;
          const int c = sl.kind == 2 ? s : j.Lc - 1 - s;
          if (fuse2(j, c, prec)) {   // the whole column step in one fused launch
            const TV in = sl.kind == 2 ? env2v(j, j.L[c], c, "xLMlma", cdt) : env2v(j, j.R[c + 1], c + 1, "yRSrse", cdt);
            const TV o = sl.kind == 2 ? env2v(j, j.L[c + 1], c + 1, "yRSrse", cdt) : env2v(j, j.R[c], c, "xLMlma", cdt);
            k2s.push_back(k2_desc(j, c, sl.kind == 2, in, o, 0, 0));
            const double f = k2_flops(k2s.back());
            k2f += f;
            j.e->flops += f;
            outs.push_back({o, sl.kind == 2 ? j.nuL + c + 1 : j.nuR + c});
            continue;
          }
          if (sl.kind == 2) {
            TV o = step2_left(st2, fin, j, c, env2v(j, j.L[c], c, "xLMlma", cdt), 0, 0, j.L[c + 1], p, q, cdt);
            outs.push_back({o, j.nuL + c + 1});
          } else {
            TV o = step2_right(st2, fin, j, c, env2v(j, j.R[c + 1], c + 1, "yRSrse", cdt), j.R[c], p, q, cdt);
            outs.push_back({o, j.nuR + c});
          }
          j.e->flops += st2.flops - f0;
        }
      }
      st1.record(rec, prec, cdt);
      st2.record(rec, prec, cdt);
      rec.tc(prec, cdt, std::move(fin));
      rec.k2(std::move(k2s), k2f);
      normalise(rec, outs);
      rec.flush(call);
    }
    for (void* p : P) scr.put(p);
    for (void* q : Q) scr.put(q);
  }
}

}  // namespace

void plan_expect(Ctx& ctx, std::vector<peps_env*>& envs, std::vector<ExpectOut>& out) {
  Arena call(&ctx.pool);
  Rec rec(&ctx, &call);
  Scratch scr(call);
  std::vector<RJob> rj;
  std::vector<R2Job> r2;
  int dtype = envs.empty() ? 0 : envs[0]->opts.dtype;
  for (peps_env* e : envs) PE_REQUIRE(e->opts.dtype == dtype, "one precision per expect call");
  const Opts& o = envs[0]->opts;
  const int prec = o.prec(), cdt = o.cdt();
  const size_t esz = dtype_size(cdt);
  const size_t budget = ctx.scratch_budget;

  // ------------------------------------------------------------ jobs ----
  // An environment with column boundaries adds the single-row sandwiches of
  // its transposed lattice and forms no two-row sandwiches.
  std::vector<std::pair<peps_env*, peps_env*>> srcs;   // (environment, owner)
  for (peps_env* e : envs) {
    srcs.push_back({e, e});
    if (e->col) srcs.push_back({e->col.get(), e});
  }
  for (const auto& src : srcs) {
    peps_env* e = src.first;
    const bool tr = src.first != src.second;
    const Lattice& L = e->lat;
    const int Lr = L.Lr, Lc = L.Lc;
    std::vector<int> rows;
    if (e->window) {
      rows.push_back(e->ci);
    } else {
      for (int r = 0; r < Lr; ++r) rows.push_back(r);
    }
    for (int r : rows) rj.push_back(make_row_job(e, src.second, tr, r, call, esz));
    std::vector<int> prs;
    if (tr || e->col) {
      // vertical bonds come from the transposed lattice
    } else if (e->window) {
      if (e->ci + 1 < Lr) prs.push_back(e->ci);
    } else {
      for (int r = 0; r + 1 < Lr; ++r) prs.push_back(r);
    }
    for (int r : prs) {
      R2Job j;
      j.e = e;
      j.r = r;
      j.Lc = Lc;
      j.T = &e->T(r - 1);
      j.B = &e->B(r + 2);
      for (int c = 0; c < Lc; ++c) {
        j.s1.push_back(&L.at(r, c));
        j.s2.push_back(&L.at(r + 1, c));
      }
      for (int c = 0; c <= Lc; ++c) {
        j.bT.push_back(j.T->bond[c]);
        j.bB.push_back(j.B->bond[c]);
        j.Dl1.push_back(c < Lc ? L.at(r, c).Dl : L.at(r, Lc - 1).Dr);
        j.Dl2.push_back(c < Lc ? L.at(r + 1, c).Dl : L.at(r + 1, Lc - 1).Dr);
      }
      j.L.assign(Lc + 1, nullptr);
      j.R.assign(Lc + 1, nullptr);
      for (int c = 0; c <= Lc; ++c) {
        j.L[c] = call.alloc(esz * env2_elems(j, c));
        j.R[c] = call.alloc(esz * env2_elems(j, c));
      }
      j.nuL = (double*)call.alloc(sizeof(double) * (Lc + 1));
      j.nuR = (double*)call.alloc(sizeof(double) * (Lc + 1));
      j.dots = (double*)call.alloc(sizeof(double) * (Lc + 1 + 3 * Lc));
      r2.push_back(std::move(j));
    }
  }

  // two-row closings: outer products of the row closings
  {
    std::vector<TcDesc> op;
    for (R2Job& j : r2) {
      const Lattice& L = j.e->lat;
      const int64_t a1 = j.Dl1[0], a2 = j.Dl2[0], b1 = j.Dl1[j.Lc], b2 = j.Dl2[j.Lc];
      op.push_back(tc_build(env2v(j, j.L[0], 0, "xLMlma", cdt), dense(L.lam[j.r + 1], cdt, "LM", {a2, a2}),
                            dense(L.lam[j.r], cdt, "lm", {a1, a1})));
      op.push_back(tc_build(env2v(j, j.R[j.Lc], j.Lc, "xLMlma", cdt), dense(L.rho[j.r + 1], cdt, "LM", {b2, b2}),
                            dense(L.rho[j.r], cdt, "lm", {b1, b1})));
    }
    rec.tc(prec, cdt, std::move(op), false);
  }

  // ------------------------------------- phase 1: column environments ----
  column_envs(rec, call, scr, rj, r2, prec, cdt, esz, budget);

  // ------------------------------------ phase 2: operator insertions ----
  // one-row: X1[c][op] (op Sz for every c, S+/S- for c < Lc-1), then X2[c][t]
  std::vector<std::vector<std::array<void*, 4>>> X1(rj.size());
  std::vector<std::vector<std::array<void*, 3>>> X2(rj.size());
  std::vector<std::vector<std::array<void*, 3>>> Y2(r2.size());
  {
    struct Item {
      int level;   // 0: X1, 1: X2, 2: two-row
      size_t job;
      int c, t;
    };
    for (int level = 0; level < 3; ++level) {
      std::vector<Item> items;
      std::vector<size_t> sz;
      if (level < 2) {
        for (size_t i = 0; i < rj.size(); ++i) {
          RJob& j = rj[i];
          if (level == 0) X1[i].assign(j.Lc, {nullptr, nullptr, nullptr, nullptr});
          else X2[i].assign(j.Lc, {nullptr, nullptr, nullptr});
          for (int c = 0; c < j.Lc; ++c) {
            if (level == 0) {
              for (int op = OP_SZ; op <= OP_SM; ++op) {
                if ((op != OP_SZ || j.tr) && c + 1 >= j.Lc) continue;
                if (j.e->window && c != j.e->cj) continue;
                X1[i][c][op] = call.alloc(esz * env_elems(j, c + 1));
                items.push_back({0, i, c, op});
                auto pq = step_scratch(j, c);
                sz.push_back(esz * (pq.first + pq.second));
              }
            } else {
              if (c + 1 >= j.Lc) continue;
              if (j.e->window && c != j.e->cj) continue;
              for (int t = 0; t < 3; ++t) {
                X2[i][c][t] = call.alloc(esz * env_elems(j, c + 2));
                items.push_back({1, i, c, t});
                auto pq = step_scratch(j, c + 1);
                sz.push_back(esz * (pq.first + pq.second));
              }
            }
          }
        }
      } else {
        for (size_t i = 0; i < r2.size(); ++i) {
          R2Job& j = r2[i];
          Y2[i].assign(j.Lc, {nullptr, nullptr, nullptr});
          for (int c = 0; c < j.Lc; ++c) {
            if (j.e->window && c != j.e->cj) continue;
            for (int t = 0; t < 3; ++t) {
              Y2[i][c][t] = call.alloc(esz * env2_elems(j, c + 1));
              items.push_back({2, i, c, t});
              auto pq = step2_scratch(j, c);
              sz.push_back(esz * (pq.first + pq.second));
            }
          }
        }
      }
      for (auto g : budget_groups(sz, budget)) {
        St st1(3, prec), st2(5, prec);
        std::vector<TcDesc> fin;
        std::vector<K2Desc> k2s;
        double k2f = 0.0;
        std::vector<void*> tmp;
        for (size_t k = g.first; k < g.second; ++k) {
          const Item& it = items[k];
          if (it.level == 2 && fuse2(r2[it.job], it.c, prec)) {   // the column step with the bond operators, fused
            R2Job& j = r2[it.job];
            k2s.push_back(k2_desc(j, it.c, true, env2v(j, j.L[it.c], it.c, "xLMlma", cdt),
                                  env2v(j, Y2[it.job][it.c][it.t], it.c + 1, "yRSrse", cdt), BOND_O1[it.t],
                                  BOND_O2[it.t]));
            const double f = k2_flops(k2s.back());
            k2f += f;
            j.e->flops += f;
            continue;
          }
          if (it.level < 2) {
            RJob& j = rj[it.job];
            auto pq = step_scratch(j, it.level == 0 ? it.c : it.c + 1);
            void* p = scr.get(esz * pq.first);
            void* q = scr.get(esz * pq.second);
            tmp.push_back(p);
            tmp.push_back(q);
            const double f0 = st1.flops;
            if (it.level == 0) {
              step_left(st1, fin, j, it.c, envv(j, j.L[it.c], it.c, "xlma", cdt), it.t, X1[it.job][it.c][it.t], p, q, cdt);
            } else {
              const int o1 = BOND_O1[it.t], o2 = BOND_O2[it.t];
              step_left(st1, fin, j, it.c + 1, envv(j, X1[it.job][it.c][o1], it.c + 1, "xlma", cdt), o2,
                        X2[it.job][it.c][it.t], p, q, cdt);
            }
            j.e->flops += st1.flops - f0;
          } else {
            R2Job& j = r2[it.job];
            auto pq = step2_scratch(j, it.c);
            void* p = scr.get(esz * pq.first);
            void* q = scr.get(esz * pq.second);
            tmp.push_back(p);
            tmp.push_back(q);
            const double f0 = st2.flops;
            step2_left(st2, fin, j, it.c, env2v(j, j.L[it.c], it.c, "xLMlma", cdt), BOND_O1[it.t], BOND_O2[it.t],
                       Y2[it.job][it.c][it.t], p, q, cdt);
            j.e->flops += st2.flops - f0;
          }
        }
        st1.record(rec, prec, cdt);
        st2.record(rec, prec, cdt);
        rec.tc(prec, cdt, std::move(fin));
        rec.k2(std::move(k2s), k2f);
        for (void* p : tmp) scr.put(p);
        rec.flush(call);
      }
    }
  }

  // ------------------------------------------------- phase 3: scalars ----
  {
    std::vector<RedDesc> rd;
    for (size_t i = 0; i < rj.size(); ++i) {
      RJob& j = rj[i];
      const int Lc = j.Lc;
      for (int c = 0; c <= Lc; ++c)
        rd.push_back(red_desc(j.L[c], j.R[c], env_elems(j, c), j.dots + c, cdt));
      for (int c = 0; c < Lc; ++c)
        if (X1[i][c][OP_SZ])
          rd.push_back(red_desc(X1[i][c][OP_SZ], j.R[c + 1], env_elems(j, c + 1), j.dots + Lc + 1 + c, cdt));
      for (int c = 0; c + 1 < Lc; ++c)
        for (int t = 0; t < 3; ++t)
          if (X2[i][c][t])
            rd.push_back(red_desc(X2[i][c][t], j.R[c + 2], env_elems(j, c + 2), j.dots + 2 * Lc + 1 + 3 * c + t, cdt));
    }
    for (size_t i = 0; i < r2.size(); ++i) {
      R2Job& j = r2[i];
      const int Lc = j.Lc;
      for (int c = 0; c <= Lc; ++c)
        rd.push_back(red_desc(j.L[c], j.R[c], env2_elems(j, c), j.dots + c, cdt));
      for (int c = 0; c < Lc; ++c)
        for (int t = 0; t < 3; ++t)
          if (Y2[i][c][t])
            rd.push_back(red_desc(Y2[i][c][t], j.R[c + 1], env2_elems(j, c + 1), j.dots + Lc + 1 + 3 * c + t, cdt));
    }
    rec.reduce(std::move(rd));
  }
  Gather g;
  std::vector<std::array<size_t, 3>> o1(rj.size());
  std::vector<std::array<size_t, 2>> o2(r2.size());
  for (size_t i = 0; i < rj.size(); ++i) {
    const size_t Lc = rj[i].Lc;
    o1[i] = {g.add(rj[i].dots, Lc + 1 + Lc + 3 * Lc), g.add(rj[i].nuL, Lc + 1), g.add(rj[i].nuR, Lc + 1)};
  }
  for (size_t i = 0; i < r2.size(); ++i) {
    const size_t Lc = r2[i].Lc;
    o2[i] = {g.add(r2[i].dots, Lc + 1 + 3 * Lc), g.add(r2[i].nuL, Lc + 1)};
  }
  g.record(rec, call);
  rec.run(call);
  g.read(ctx.stream);

  // ------------------------------------------------- host arithmetic ----
  out.assign(envs.size(), ExpectOut());
  std::unordered_map<peps_env*, size_t> pos;
  for (size_t i = 0; i < envs.size(); ++i) {
    pos[envs[i]] = i;
    const Lattice& L = envs[i]->lat;
    ExpectOut& eo = out[i];
    if (envs[i]->window) {
      eo.sz.assign(1, NAN);
      eo.bond.assign(2, NAN);
    } else {
      eo.sz.assign((size_t)L.Lr * L.Lc, NAN);
      eo.bond.assign((size_t)L.Lr * (L.Lc - 1) + (size_t)(L.Lr - 1) * L.Lc, NAN);
    }
    eo.log_norm = NAN;
  }
  std::vector<std::vector<double>> hdots(rj.size()), hnuL(rj.size()), hnuR(rj.size());
  std::vector<std::vector<double>> h2dots(r2.size()), h2nuL(r2.size());
  for (size_t i = 0; i < rj.size(); ++i) {
    const size_t Lc = rj[i].Lc;
    hdots[i] = g.slice(o1[i][0], Lc + 1 + Lc + 3 * Lc);
    hnuL[i] = g.slice(o1[i][1], Lc + 1);
    hnuR[i] = g.slice(o1[i][2], Lc + 1);
  }
  for (size_t i = 0; i < r2.size(); ++i) {
    const size_t Lc = r2[i].Lc;
    h2dots[i] = g.slice(o2[i][0], Lc + 1 + 3 * Lc);
    h2nuL[i] = g.slice(o2[i][1], Lc + 1);
  }
  for (size_t i = 0; i < rj.size(); ++i) {
    const RJob& j = rj[i];
    peps_env* e = j.e;
    ExpectOut& eo = out[pos[j.owner]];
    const int Lc = j.Lc, Lr = e->lat.Lr;
    const std::vector<double>& D = hdots[i];
    const std::vector<double>& nu = hnuL[i];
    for (int c = 0; c < Lc; ++c) {
      if (j.tr || !X1[i][c][OP_SZ]) continue;
      const double v = D[Lc + 1 + c] / (std::sqrt(nu[c + 1]) * D[c + 1]);
      if (e->window) {
        if (c == e->cj && j.r == e->ci) eo.sz[0] = v;
      } else {
        eo.sz[(size_t)j.r * Lc + c] = v;
      }
    }
    for (int c = 0; c + 1 < Lc; ++c) {
      if (!X2[i][c][0]) continue;
      double num = 0.0;
      for (int t = 0; t < 3; ++t) num += BOND_W[t] * D[2 * Lc + 1 + 3 * c + t];
      const double v = num / (std::sqrt(nu[c + 1] * nu[c + 2]) * D[c + 2]);
      if (j.tr && e->window) {
        // the transposed window's centre bond to the right is the centre's bond downwards
        if (c == e->cj && j.r == e->ci) eo.bond[1] = v;
      } else if (j.tr) {
        // bond (j.r, c)-(j.r, c+1) of the transpose is the vertical bond (c, j.r)-(c+1, j.r)
        eo.bond[(size_t)Lc * (Lr - 1) + (size_t)c * Lr + j.r] = v;
      } else if (e->window) {
        if (c == e->cj && j.r == e->ci) eo.bond[0] = v;
      } else {
        eo.bond[(size_t)j.r * (Lc - 1) + c] = v;
      }
    }
    if (!j.tr && j.r == Lr / 2) {
      const int cc = Lc / 2;
      double lg = e->Tlog(j.r - 1) + e->Blog(j.r + 1) + std::log(std::fabs(D[cc]));
      for (int k = 1; k <= cc; ++k) lg += 0.5 * std::log(nu[k]);
      for (int k = cc; k < Lc; ++k) lg += 0.5 * std::log(hnuR[i][k]);
      eo.log_norm = lg;
      eo.sign = D[cc] < 0 ? -1.0 : 1.0;
    }
  }
  for (size_t i = 0; i < r2.size(); ++i) {
    const R2Job& j = r2[i];
    peps_env* e = j.e;
    ExpectOut& eo = out[pos[e]];
    const int Lc = j.Lc;
    const std::vector<double>& D = h2dots[i];
    const std::vector<double>& nu = h2nuL[i];
    for (int c = 0; c < Lc; ++c) {
      if (!Y2[i][c][0]) continue;
      double num = 0.0;
      for (int t = 0; t < 3; ++t) num += BOND_W[t] * D[Lc + 1 + 3 * c + t];
      const double v = num / (std::sqrt(nu[c + 1]) * D[c + 1]);
      if (e->window) {
        if (c == e->cj && j.r == e->ci) eo.bond[1] = v;
      } else {
        eo.bond[(size_t)e->lat.Lr * (Lc - 1) + (size_t)j.r * Lc + c] = v;
      }
    }
  }
}

}  // namespace pe

namespace pe {

namespace {

// The single-row sandwich jobs of (environment, row) pairs with their left
// and right column environments.  An environment is immutable, so these
// are computed once, in the environment's own memory, and kept with it for
// later site, bond and fit calls; jid[i] indexes the job of keys[i].
void row_sandwiches(Ctx& ctx, Rec& rec, Arena& call, Scratch& scr, const std::vector<std::pair<peps_env*, int>>& keys,
                    std::vector<RJob>& rj, std::vector<size_t>& jid, int prec, int cdt) {
  const size_t esz = dtype_size(cdt);
  std::map<std::pair<peps_env*, int>, size_t> job_of;
  std::vector<RJob> fresh;
  std::vector<size_t> fresh_at;
  // the new sandwiches' buffers: one arena per environment, handed to the
  // environment only once the sandwiches exist (released if they fail)
  std::map<peps_env*, std::unique_ptr<Arena>> held;
  for (size_t i = 0; i < keys.size(); ++i) {
    auto it = job_of.find(keys[i]);
    if (it == job_of.end()) {
      it = job_of.emplace(keys[i], rj.size()).first;
      peps_env* e = keys[i].first;
      auto c = e->row_env.find(keys[i].second);
      if (c != e->row_env.end()) {
        rj.push_back(*static_cast<const RJob*>(c->second.get()));
      } else {
        auto& a = held[e];
        if (!a) a = std::make_unique<Arena>(&e->ctx->pool);
        fresh.push_back(make_row_job(e, e, false, keys[i].second, *a, esz));
        fresh_at.push_back(rj.size());
        rj.push_back(fresh.back());
      }
    }
    jid[i] = it->second;
  }
  if (fresh.empty()) return;
  std::vector<R2Job> r2;
  column_envs(rec, call, scr, fresh, r2, prec, cdt, esz, ctx.scratch_budget);
  for (auto& h : held) h.first->arena.adopt(*h.second);
  for (size_t k = 0; k < fresh.size(); ++k) {
    const RJob& j = fresh[k];
    j.e->row_env[j.r] = std::make_shared<RJob>(j);
    rj[fresh_at[k]] = j;
  }
}

}  // namespace

void plan_site_env(Ctx& ctx, std::vector<SiteReq>& req, std::vector<double>& log_z, std::vector<double>& sign,
                   double& flops) {
  Arena call(&ctx.pool);
  Rec rec(&ctx, &call);
  Scratch scr(call);
  const Opts& o = req[0].e->opts;
  for (const SiteReq& q : req) PE_REQUIRE(q.e->opts.dtype == o.dtype, "one precision per site-environment call");
  const int prec = o.prec(), cdt = o.cdt();
  const size_t esz = dtype_size(cdt);

  // one single-row sandwich per distinct (environment, row)
  std::vector<RJob> rj;
  std::vector<size_t> jid(req.size());
  {
    std::vector<std::pair<peps_env*, int>> keys;
    for (const auto& q : req) keys.push_back({q.e, q.r});
    row_sandwiches(ctx, rec, call, scr, keys, rj, jid, prec, cdt);
  }

  // N[l,u,r,d,m,v,s,g] = L[c][x,l,m,a] T[c][a,u,v,e] B[c][x,d,g,y] R[c+1][y,r,s,e]
  // (the norm network of the row with site c's ket and bra taken out):
  // three grouped stages per budget group, N in the compute dtype
  std::vector<void*> raw(req.size());
  std::vector<int64_t> nel(req.size());
  std::vector<size_t> sz(req.size());
  struct Dims {
    int64_t x, y, a, e, Dl, Du, Dr, Dd;
  };
  std::vector<Dims> dm(req.size());
  for (size_t i = 0; i < req.size(); ++i) {
    const RJob& j = rj[jid[i]];
    const int c = req[i].c;
    Dims d{j.bB[c], j.bB[c + 1], j.bT[c], j.bT[c + 1], j.Dl[c], j.T->leg[c], j.Dl[c + 1], j.B->leg[c]};
    dm[i] = d;
    nel[i] = d.Dl * d.Du * d.Dr * d.Dd * d.Dl * d.Du * d.Dr * d.Dd;
    raw[i] = cdt == DT_F64 ? (void*)req[i].out : call.alloc(esz * nel[i]);
    sz[i] = esz * (size_t)(d.x * d.Dl * d.Dl * d.Du * d.Du * d.e + d.Dl * d.Dl * d.Du * d.Du * d.e * d.Dd * d.Dd * d.y);
  }
  flops = 0.0;
  std::vector<RedDesc> rd;
  for (auto g : budget_groups(sz, ctx.scratch_budget)) {
    std::vector<TcDesc> s1, s2, s3;
    std::vector<void*> tmp;
    for (size_t i = g.first; i < g.second; ++i) {
      const RJob& j = rj[jid[i]];
      const int c = req[i].c;
      const Dims& d = dm[i];
      void* p = scr.get(esz * d.x * d.Dl * d.Dl * d.Du * d.Du * d.e);
      void* q = scr.get(esz * d.Dl * d.Dl * d.Du * d.Du * d.e * d.Dd * d.Dd * d.y);
      tmp.push_back(p);
      tmp.push_back(q);
      TV L = envv(j, j.L[c], c, "xlma", cdt);
      TV T = dense(j.T->tc[c], cdt, "auve", {d.a, d.Du, d.Du, d.e});
      TV B = dense(j.B->tc[c], cdt, "xdgy", {d.x, d.Dd, d.Dd, d.y});
      TV R = envv(j, j.R[c + 1], c + 1, "yrse", cdt);
      // intermediate leg orders chosen so that every index group of each
      // contraction merges into at most four strided sub-dimensions; on a
      // transposed lattice N is written in the original site's leg order
      // (l, u, r, d) = (u, l, d, r) of the transpose
      const bool tr = req[i].tr;
      TV y1 = tr ? dense(p, cdt, "xulvme", {d.x, d.Du, d.Dl, d.Du, d.Dl, d.e})
                 : dense(p, cdt, "xlumve", {d.x, d.Dl, d.Du, d.Dl, d.Du, d.e});
      TV y2 = tr ? dense(q, cdt, "uldvmgye", {d.Du, d.Dl, d.Dd, d.Du, d.Dl, d.Dd, d.y, d.e})
                 : dense(q, cdt, "ludmvgye", {d.Dl, d.Du, d.Dd, d.Dl, d.Du, d.Dd, d.y, d.e});
      TV n = tr ? dense(raw[i], cdt, "uldrvmgs", {d.Du, d.Dl, d.Dd, d.Dr, d.Du, d.Dl, d.Dd, d.Dr})
                : dense(raw[i], cdt, "lurdmvsg", {d.Dl, d.Du, d.Dr, d.Dd, d.Dl, d.Du, d.Dr, d.Dd});
      s1.push_back(tc_build(y1, L, T));
      s2.push_back(tc_build(y2, y1, B));
      s3.push_back(tc_build(n, y2, R));
      flops += tc_flops(s1.back()) + tc_flops(s2.back()) + tc_flops(s3.back());
    }
    rec.tc(prec, cdt, std::move(s1));
    rec.tc(prec, cdt, std::move(s2));
    rec.tc(prec, cdt, std::move(s3));
    for (void* p : tmp) scr.put(p);
    rec.flush(call);
  }
  // <L[c+1], R[c+1]>: with the left step's squared norm, the value of A N A
  for (size_t i = 0; i < req.size(); ++i) {
    const RJob& j = rj[jid[i]];
    const int c = req[i].c;
    rd.push_back(red_desc(j.L[c + 1], j.R[c + 1], env_elems(j, c + 1), j.dots + c + 1, cdt));
  }
  rec.reduce(std::move(rd));
  std::vector<std::vector<double>> hd, hl, hr;
  run_and_read_dots(rec, call, rj, ctx.stream, hd, hl, hr);
  log_z.assign(req.size(), 0.0);
  sign.assign(req.size(), 1.0);
  double* w2 = (double*)call.alloc(sizeof(double) * req.size());
  std::vector<EwDesc> fill, scale;
  for (size_t i = 0; i < req.size(); ++i) {
    const RJob& j = rj[jid[i]];
    peps_env* e = req[i].e;
    const int c = req[i].c, r = req[i].r;
    const double w = std::sqrt(hl[jid[i]][c + 1]) * hd[jid[i]][c + 1];
    if (!(std::isfinite(w) && w != 0.0))
      throw Error(ST_NONFINITE, "site environment (" + std::to_string(r) + "," + std::to_string(c) + ") has A N A = " +
                                    std::to_string(w));
    double lg = e->Tlog(r - 1) + e->Blog(r + 1) + std::log(std::fabs(w));
    for (int k = 1; k <= c; ++k) lg += 0.5 * std::log(hl[jid[i]][k]);
    for (int k = c + 1; k < j.Lc; ++k) lg += 0.5 * std::log(hr[jid[i]][k]);
    log_z[i] = lg;
    sign[i] = w < 0 ? -1.0 : 1.0;
    EwDesc f = ew_desc(EW_FILL, nullptr, DT_F64, w2 + i, DT_F64, 1);
    f.a = w * w;
    fill.push_back(f);
    EwDesc s = ew_desc(EW_RSQRT, raw[i], cdt, req[i].out, DT_F64, nel[i]);
    s.sptr = w2 + i;
    scale.push_back(s);
  }
  Rec rec2(&ctx, &call);
  rec2.ew(fill);
  rec2.ew(scale);
  rec2.run(call);
  dev::sync(ctx.stream);
}

}  // namespace pe

namespace pe {

void plan_bond_env(Ctx& ctx, std::vector<BondReq>& req, double& flops) {
  Arena call(&ctx.pool);
  Rec rec(&ctx, &call);
  Scratch scr(call);
  const Opts& o = req[0].e->opts;
  for (const BondReq& q : req) PE_REQUIRE(q.e->opts.dtype == o.dtype, "one precision per bond-environment call");
  const int prec = o.prec(), cdt = o.cdt();
  const size_t esz = dtype_size(cdt);

  std::vector<RJob> rj;
  std::vector<size_t> jid(req.size());
  {
    std::vector<std::pair<peps_env*, int>> keys;
    for (const auto& q : req) keys.push_back({q.e, q.r});
    row_sandwiches(ctx, rec, call, scr, keys, rj, jid, prec, cdt);
  }

  // gates in the compute dtype
  std::vector<const void*> gate(req.size());
  {
    std::vector<EwDesc> cv;
    for (size_t i = 0; i < req.size(); ++i) {
      const int64_t d = rj[jid[i]].s[req[i].c]->d;
      if (cdt == DT_F64) {
        gate[i] = req[i].gate;
      } else {
        void* g = call.alloc(esz * d * d * d * d);
        cv.push_back(ew_desc(EW_COPY, req[i].gate, DT_F64, g, cdt, d * d * d * d));
        gate[i] = g;
      }
    }
    if (!cv.empty()) rec.ew(std::move(cv));
  }

  // Per bond (c, c+1) of row r:
  //   X[l,u,d,m,v,g,y,e]  = L[c] T[c] B[c]
  //   Z[R,S,e,U,V,y,D,G]  = R[c+2] T[c+1] B[c+1]
  //   Th[p,P,l,u,d,U,R,D] = gate[p,P,q,Q] A_c[q,l,u,r,d] A_c+1[Q,r,U,R,D]
  //   b_left  = X . ((Z . A_c+1 bra) . Th)   (the right block takes its bra first)
  //   b_right = ((X . A_c bra) . Th) . Z     (the left block takes its bra first)
  // so that no intermediate carries both bra tensors' open legs (the pair
  // environment would cost D^6 chi^2 d^2 entries per bond).  Leg orders are
  // chosen so that every index group of each contraction merges into at
  // most four strided sub-dimensions.
  struct Dims {
    int64_t d, x, y, z, a, e, f, Dl, Du, Dd, R, U, D;
  };
  std::vector<Dims> dm(req.size());
  std::vector<size_t> sz(req.size());
  std::vector<void*> rawl(req.size(), nullptr), rawr(req.size(), nullptr);
  for (size_t i = 0; i < req.size(); ++i) {
    const RJob& j = rj[jid[i]];
    const int c = req[i].c;
    const Site& s1 = *j.s[c];
    const Site& s2 = *j.s[c + 1];
    PE_REQUIRE(s1.d == s2.d, "the two sites of a gated bond need one physical dimension");
    Dims q{s1.d, j.bB[c], j.bB[c + 1], j.bB[c + 2], j.bT[c], j.bT[c + 1], j.bT[c + 2],
           j.Dl[c], j.T->leg[c], j.B->leg[c], j.Dl[c + 2], j.T->leg[c + 1], j.B->leg[c + 1]};
    dm[i] = q;
    const int64_t K1 = q.Dl * q.Du * j.Dl[c + 1] * q.Dd, K2 = j.Dl[c + 1] * q.U * q.R * q.D;
    if (req[i].bl) rawl[i] = cdt == DT_F64 ? (void*)req[i].bl : call.alloc(esz * q.d * K1);
    if (req[i].br) rawr[i] = cdt == DT_F64 ? (void*)req[i].br : call.alloc(esz * q.d * K2);
    const int64_t n = q.x * q.Dl * q.Du * q.Dl * q.Du * q.e                 // X1
                      + q.Dl * q.Du * q.Dd * q.Dl * q.Du * q.Dd * q.y * q.e   // X
                      + q.z * q.R * q.R * q.e * q.U * q.U                     // Z1
                      + q.R * q.R * q.e * q.U * q.U * q.y * q.D * q.D         // Z
                      + 2 * q.d * q.d * q.Dl * q.Du * q.Dd * q.U * q.R * q.D   // A_c A_c+1, Th
                      + 2 * q.R * q.e * q.U * q.y * q.D * q.d * j.Dl[c + 1]   // Zb, Wr
                      + 2 * q.Dl * q.Du * q.Dd * q.y * q.e * q.d * j.Dl[c + 1];   // Xb, Wl
    sz[i] = esz * (size_t)n;
  }
  flops = 0.0;
  for (auto g : budget_groups(sz, ctx.scratch_budget)) {
    std::vector<TcDesc> st[5];
    std::vector<void*> tmp;
    auto add = [&](int k, const TcDesc& t) {
      st[k].push_back(t);
      flops += tc_flops(t);
    };
    for (size_t i = g.first; i < g.second; ++i) {
      const RJob& j = rj[jid[i]];
      const int c = req[i].c;
      const Dims& q = dm[i];
      const int64_t h = j.Dl[c + 1];
      auto get = [&](int64_t n) {
        void* p = scr.get(esz * n);
        tmp.push_back(p);
        return p;
      };
      TV L = envv(j, j.L[c], c, "xlma", cdt);
      TV T1 = dense(j.T->tc[c], cdt, "auve", {q.a, q.Du, q.Du, q.e});
      TV B1 = dense(j.B->tc[c], cdt, "xdgy", {q.x, q.Dd, q.Dd, q.y});
      TV T2 = dense(j.T->tc[c + 1], cdt, "eUVf", {q.e, q.U, q.U, q.f});
      TV B2 = dense(j.B->tc[c + 1], cdt, "yDGz", {q.y, q.D, q.D, q.z});
      TV R = envv(j, j.R[c + 2], c + 2, "zRSf", cdt);
      TV G = dense(gate[i], cdt, "pPqQ", {q.d, q.d, q.d, q.d});
      TV x1 = dense(get(q.x * q.Dl * q.Du * q.Dl * q.Du * q.e), cdt, "xlumve", {q.x, q.Dl, q.Du, q.Dl, q.Du, q.e});
      TV X = dense(get(q.Dl * q.Du * q.Dd * q.Dl * q.Du * q.Dd * q.y * q.e), cdt, "ludmvgye",
                   {q.Dl, q.Du, q.Dd, q.Dl, q.Du, q.Dd, q.y, q.e});
      TV z1 = dense(get(q.z * q.R * q.R * q.e * q.U * q.U), cdt, "zRSeUV", {q.z, q.R, q.R, q.e, q.U, q.U});
      TV Z = dense(get(q.R * q.R * q.e * q.U * q.U * q.y * q.D * q.D), cdt, "RSeUVyDG",
                   {q.R, q.R, q.e, q.U, q.U, q.y, q.D, q.D});
      TV aa = dense(get(q.d * q.d * q.Dl * q.Du * q.Dd * q.U * q.R * q.D), cdt, "qQludURD",
                    {q.d, q.d, q.Dl, q.Du, q.Dd, q.U, q.R, q.D});
      TV th = dense(get(q.d * q.d * q.Dl * q.Du * q.Dd * q.U * q.R * q.D), cdt, "pPludURD",
                    {q.d, q.d, q.Dl, q.Du, q.Dd, q.U, q.R, q.D});
      const Site& s1 = *j.s[c];
      const Site& s2 = *j.s[c + 1];
      add(0, tc_build(x1, L, T1));
      add(0, tc_build(z1, R, T2));
      add(0, tc_build(aa, site_tv(s1, OP_ID, false, cdt, "qlurd"), site_tv(s2, OP_ID, false, cdt, "QrURD")));
      add(1, tc_build(X, x1, B1));
      add(1, tc_build(Z, z1, B2));
      add(1, tc_build(th, G, aa));
      // on a transposed lattice b is written in the original site's leg
      // order (l, u, r, d) = (u, l, d, r) of the transpose
      const bool tr = req[i].tr;
      if (rawl[i]) {
        TV zb = dense(get(q.R * q.e * q.U * q.y * q.D * q.d * h), cdt, "ReUyDPs", {q.R, q.e, q.U, q.y, q.D, q.d, h});
        TV wl = dense(get(q.e * q.y * h * q.d * q.Dl * q.Du * q.Dd), cdt, "eysplud", {q.e, q.y, h, q.d, q.Dl, q.Du, q.Dd});
        add(2, tc_build(zb, Z, site_tv(s2, OP_ID, false, cdt, "PsVSG")));
        add(3, tc_build(wl, zb, th));
        add(4, tc_build(tr ? dense(rawl[i], cdt, "pvmgs", {q.d, q.Du, q.Dl, q.Dd, h})
                           : dense(rawl[i], cdt, "pmvsg", {q.d, q.Dl, q.Du, h, q.Dd}),
                        X, wl));
      }
      if (rawr[i]) {
        TV xb = dense(get(q.Dl * q.Du * q.Dd * q.y * q.e * q.d * h), cdt, "ludyeps", {q.Dl, q.Du, q.Dd, q.y, q.e, q.d, h});
        TV wr = dense(get(h * q.d * q.R * q.e * q.U * q.y * q.D), cdt, "sPReUyD", {h, q.d, q.R, q.e, q.U, q.y, q.D});
        add(2, tc_build(xb, X, site_tv(s1, OP_ID, false, cdt, "pmvsg")));
        add(3, tc_build(wr, xb, th));
        add(4, tc_build(tr ? dense(rawr[i], cdt, "PVsGS", {q.d, q.U, h, q.D, q.R})
                           : dense(rawr[i], cdt, "PsVSG", {q.d, h, q.U, q.R, q.D}),
                        wr, Z));
      }
    }
    for (int k = 0; k < 5; ++k) rec.tc(prec, cdt, std::move(st[k]));
    for (void* p : tmp) scr.put(p);
    rec.flush(call);
  }
  // <L[k], R[k]> at k = c+1, c+2 (once per job and column)
  {
    std::vector<RedDesc> rd;
    std::vector<std::vector<char>> done(rj.size());
    for (size_t k = 0; k < rj.size(); ++k) done[k].assign(rj[k].Lc + 1, 0);
    for (size_t i = 0; i < req.size(); ++i) {
      const RJob& j = rj[jid[i]];
      for (int k = req[i].c + 1; k <= req[i].c + 2; ++k) {
        if (done[jid[i]][k]) continue;
        done[jid[i]][k] = 1;
        rd.push_back(red_desc(j.L[k], j.R[k], env_elems(j, k), j.dots + k, cdt));
      }
    }
    rec.reduce(std::move(rd));
  }
  std::vector<std::vector<double>> hd, hl, hr;
  run_and_read_dots(rec, call, rj, ctx.stream, hd, hl, hr);
  // b_left / (sqrt(nuR[c+1]) |w_c|), b_right / (sqrt(nuL[c+1]) |w_c+1|), with
  // w_k = sqrt(nuL[k+1]) <L[k+1], R[k+1]> (= sum_p A N A of site k): the
  // scaling of the sites' norm environments
  double* s2 = (double*)call.alloc(sizeof(double) * 2 * req.size());
  std::vector<EwDesc> fill, scale;
  for (size_t i = 0; i < req.size(); ++i) {
    const size_t k = jid[i];
    const int c = req[i].c;
    const double w0 = std::sqrt(hl[k][c + 1]) * hd[k][c + 1], w1 = std::sqrt(hl[k][c + 2]) * hd[k][c + 2];
    const double sl = std::sqrt(hr[k][c + 1]) * std::fabs(w0), sr = std::sqrt(hl[k][c + 1]) * std::fabs(w1);
    if (!(std::isfinite(sl) && sl > 0.0 && std::isfinite(sr) && sr > 0.0))
      throw Error(ST_NONFINITE, "bond environment (" + std::to_string(req[i].r) + "," + std::to_string(c) +
                                    ") has a zero or non-finite scale");
    const Dims& q = dm[i];
    const int64_t h = rj[k].Dl[c + 1];
    for (int side = 0; side < 2; ++side) {
      void* raw = side == 0 ? rawl[i] : rawr[i];
      if (!raw) continue;
      EwDesc f = ew_desc(EW_FILL, nullptr, DT_F64, s2 + 2 * i + side, DT_F64, 1);
      f.a = side == 0 ? sl * sl : sr * sr;
      fill.push_back(f);
      const int64_t n = side == 0 ? q.d * q.Dl * q.Du * h * q.Dd : q.d * h * q.U * q.R * q.D;
      EwDesc e = ew_desc(EW_RSQRT, raw, cdt, side == 0 ? req[i].bl : req[i].br, DT_F64, n);
      e.sptr = s2 + 2 * i + side;
      scale.push_back(e);
    }
  }
  Rec rec2(&ctx, &call);
  rec2.ew(fill);
  rec2.ew(scale);
  rec2.run(call);
  dev::sync(ctx.stream);
}

}  // namespace pe

namespace pe {

void plan_overlap(Ctx& ctx, std::vector<OvReq>& req) {
  Arena call(&ctx.pool);
  Rec rec(&ctx, &call);
  // three chains per request: <X|Y>, <X|X>, <Y|Y>; E_{c+1}[z,w] = E_c[x,y] X_c[x,k,b,z] Y_c[y,k,b,w]
  struct Chain {
    const Mps* x;
    const Mps* y;
    double* e[2];
    double* tmp;
  };
  std::vector<Chain> ch;
  int maxLc = 0;
  std::vector<EwDesc> init;
  for (const OvReq& q : req)
    for (int t = 0; t < 3; ++t) {
      Chain c;
      c.x = t == 2 ? q.y : q.x;
      c.y = t == 1 ? q.x : q.y;
      const int Lc = (int)c.x->leg.size();
      maxLc = std::max(maxLc, Lc);
      int64_t me = 1, mt = 1;
      for (int k = 0; k <= Lc; ++k) me = std::max(me, (int64_t)c.x->bond[k] * c.y->bond[k]);
      for (int k = 0; k < Lc; ++k)
        mt = std::max(mt, (int64_t)c.y->bond[k] * c.x->leg[k] * c.x->leg[k] * c.x->bond[k + 1]);
      c.e[0] = (double*)call.alloc(sizeof(double) * me);
      c.e[1] = (double*)call.alloc(sizeof(double) * me);
      c.tmp = (double*)call.alloc(sizeof(double) * mt);
      EwDesc f = ew_desc(EW_FILL, nullptr, DT_F64, c.e[0], DT_F64, 1);
      f.a = 1.0;
      init.push_back(f);
      ch.push_back(c);
    }
  rec.ew(std::move(init));
  for (int s = 0; s < maxLc; ++s) {
    std::vector<TcDesc> st1, st2;
    for (Chain& c : ch) {
      if (s >= (int)c.x->leg.size()) continue;
      const int64_t bx = c.x->bond[s], by = c.y->bond[s], bx1 = c.x->bond[s + 1], by1 = c.y->bond[s + 1];
      const int64_t l = c.x->leg[s];
      TV E = dense(c.e[s & 1], DT_F64, "xy", {bx, by});
      TV X = dense(c.x->t64[s], DT_F64, "xkbz", {bx, l, l, bx1});
      TV Y = dense(c.y->t64[s], DT_F64, "ykbw", {by, l, l, by1});
      TV y1 = dense(c.tmp, DT_F64, "ykbz", {by, l, l, bx1});
      st1.push_back(tc_build(y1, E, X));
      st2.push_back(tc_build(dense(c.e[(s + 1) & 1], DT_F64, "zw", {bx1, by1}), y1, Y));
    }
    rec.tc(TP_F64, DT_F64, std::move(st1));
    rec.tc(TP_F64, DT_F64, std::move(st2));
    rec.flush(call);
  }
  Gather g;
  for (size_t i = 0; i < req.size(); ++i)
    for (int t = 0; t < 3; ++t) {
      const Chain& c = ch[3 * i + t];
      g.add((const double*)c.e[c.x->leg.size() & 1], 1);
    }
  g.record(rec, call);
  rec.run(call);
  g.read(ctx.stream);
  for (size_t i = 0; i < req.size(); ++i)
    for (int t = 0; t < 3; ++t) req[i].out[t] = g.host[3 * i + t];
}

}  // namespace pe

namespace pe {

namespace {

// One raw column step with explicit ket and bra views (no normalisation).
void step_tv(St& st, std::vector<TcDesc>& fin, const RJob& j, int c, bool left, const TV& in, const TV& ket,
             const TV& bra, void* out, void* P, void* Q, int cdt) {
  TV T = dense(j.T->tc[c], cdt, "auve", {j.bT[c], j.T->leg[c], j.T->leg[c], j.bT[c + 1]});
  TV B = dense(j.B->tc[c], cdt, "xdgy", {j.bB[c], j.B->leg[c], j.B->leg[c], j.bB[c + 1]});
  if (left) {
    TV y3 = chain_left(st, in, T, ket, bra, P, Q, cdt);
    fin.push_back(tc_build(envv(j, out, c + 1, "yrse", cdt), y3, B));
  } else {
    TV y3 = chain_right(st, in, T, ket, bra, P, Q, cdt);
    fin.push_back(tc_build(envv(j, out, c, "xlma", cdt), y3, B));
  }
  st.flops += tc_flops(fin.back());
}

}  // namespace

void plan_bond_fit(Ctx& ctx, std::vector<FitReq>& req, double& flops) {
  Arena call(&ctx.pool);
  Rec rec(&ctx, &call);
  Scratch scr(call);
  const Opts& o = req[0].e->opts;
  for (const FitReq& q : req) PE_REQUIRE(q.e->opts.dtype == o.dtype, "one precision per bond-fit call");
  PE_REQUIRE(o.cdt() == DT_F64, "the bond fit takes float64 substitutes: it needs a float64 environment");
  const int prec = o.prec(), cdt = DT_F64;
  const size_t esz = sizeof(double);

  std::vector<RJob> rj;
  std::vector<size_t> jid(req.size());
  {
    std::vector<std::pair<peps_env*, int>> keys;
    for (const auto& q : req) keys.push_back({q.e, q.r});
    row_sandwiches(ctx, rec, call, scr, keys, rj, jid, prec, cdt);
  }
  flops = 0.0;

  // the substitutes as site views (same shape and storage order as the sites)
  std::vector<Site> v1(req.size()), v2(req.size());
  for (size_t i = 0; i < req.size(); ++i) {
    const RJob& j = rj[jid[i]];
    v1[i] = *j.s[req[i].c];
    v2[i] = *j.s[req[i].c + 1];
    v1[i].op[0] = const_cast<double*>(req[i].s1);
    v2[i].op[0] = const_cast<double*>(req[i].s2);
  }
  // raw environments with the substitutes: R1 = step(R[c+2]; S2), L2 = step(L[c]; S1)
  std::vector<void*> R1(req.size()), L2(req.size());
  {
    St st(3, prec);
    std::vector<TcDesc> fin;
    std::vector<void*> tmp;
    for (size_t i = 0; i < req.size(); ++i) {
      const RJob& j = rj[jid[i]];
      const int c = req[i].c;
      R1[i] = call.alloc(esz * env_elems(j, c + 1));
      L2[i] = call.alloc(esz * env_elems(j, c + 1));
      for (int k = 0; k < 2; ++k) {
        const int cc = k == 0 ? c + 1 : c;
        auto pq = step_scratch(j, cc);
        void* P = scr.get(esz * pq.first);
        void* Q = scr.get(esz * pq.second);
        tmp.push_back(P);
        tmp.push_back(Q);
        const Site& v = k == 0 ? v2[i] : v1[i];
        if (k == 0)
          step_tv(st, fin, j, cc, false, envv(j, j.R[c + 2], c + 2, "yrse", cdt), site_tv(v, OP_ID, false, cdt, "plurd"),
                  site_tv(v, OP_ID, false, cdt, "pmvsg"), R1[i], P, Q, cdt);
        else
          step_tv(st, fin, j, cc, true, envv(j, j.L[c], c, "xlma", cdt), site_tv(v, OP_ID, false, cdt, "plurd"),
                  site_tv(v, OP_ID, false, cdt, "pmvsg"), L2[i], P, Q, cdt);
      }
    }
    st.record(rec, prec, cdt);
    rec.tc(prec, cdt, std::move(fin));
    flops += st.flops;
    for (void* p : tmp) scr.put(p);
    rec.flush(call);
  }

  // b1 and b2 (as for the gated bond, the substitutes as the bras),
  // N1 = L[c] T B R1, N2 = L2 T B R[c+2]; leg orders as in the site and bond
  // environments (the transposed forms write the sites' own order)
  for (size_t i = 0; i < req.size(); ++i) {
    const RJob& j = rj[jid[i]];
    const int c = req[i].c;
    const bool tr = req[i].tr;
    const int64_t d = j.s[c]->d;
    const int64_t x = j.bB[c], y = j.bB[c + 1], z = j.bB[c + 2], a = j.bT[c], e = j.bT[c + 1], f = j.bT[c + 2];
    const int64_t Dl = j.Dl[c], Du = j.T->leg[c], Dd = j.B->leg[c], h = j.Dl[c + 1];
    const int64_t R = j.Dl[c + 2], U = j.T->leg[c + 1], D = j.B->leg[c + 1];
    std::vector<TcDesc> st[5];
    std::vector<void*> tmp;
    auto add = [&](int k, const TcDesc& t) {
      st[k].push_back(t);
      flops += tc_flops(t);
    };
    auto get = [&](int64_t n) {
      void* p = scr.get(esz * n);
      tmp.push_back(p);
      return p;
    };
    TV L = envv(j, j.L[c], c, "xlma", cdt);
    TV T1 = dense(j.T->tc[c], cdt, "auve", {a, Du, Du, e});
    TV B1 = dense(j.B->tc[c], cdt, "xdgy", {x, Dd, Dd, y});
    TV T2 = dense(j.T->tc[c + 1], cdt, "eUVf", {e, U, U, f});
    TV B2 = dense(j.B->tc[c + 1], cdt, "yDGz", {y, D, D, z});
    TV Rr = envv(j, j.R[c + 2], c + 2, "zRSf", cdt);
    TV G = dense(req[i].gate, cdt, "pPqQ", {d, d, d, d});
    TV x1 = dense(get(x * Dl * Du * Dl * Du * e), cdt, "xlumve", {x, Dl, Du, Dl, Du, e});
    TV X = dense(get(Dl * Du * Dd * Dl * Du * Dd * y * e), cdt, "ludmvgye", {Dl, Du, Dd, Dl, Du, Dd, y, e});
    TV z1 = dense(get(z * R * R * e * U * U), cdt, "zRSeUV", {z, R, R, e, U, U});
    TV Z = dense(get(R * R * e * U * U * y * D * D), cdt, "RSeUVyDG", {R, R, e, U, U, y, D, D});
    TV aa = dense(get(d * d * Dl * Du * Dd * U * R * D), cdt, "qQludURD", {d, d, Dl, Du, Dd, U, R, D});
    TV th = dense(get(d * d * Dl * Du * Dd * U * R * D), cdt, "pPludURD", {d, d, Dl, Du, Dd, U, R, D});
    TV zb = dense(get(R * e * U * y * D * d * h), cdt, "ReUyDPs", {R, e, U, y, D, d, h});
    TV wl = dense(get(e * y * h * d * Dl * Du * Dd), cdt, "eysplud", {e, y, h, d, Dl, Du, Dd});
    TV xb = dense(get(Dl * Du * Dd * y * e * d * h), cdt, "ludyeps", {Dl, Du, Dd, y, e, d, h});
    TV wr = dense(get(h * d * R * e * U * y * D), cdt, "sPReUyD", {h, d, R, e, U, y, D});
    add(0, tc_build(x1, L, T1));
    add(0, tc_build(z1, Rr, T2));
    add(0, tc_build(aa, site_tv(*j.s[c], OP_ID, false, cdt, "qlurd"), site_tv(*j.s[c + 1], OP_ID, false, cdt, "QrURD")));
    add(1, tc_build(X, x1, B1));
    add(1, tc_build(Z, z1, B2));
    add(1, tc_build(th, G, aa));
    // b1 = X . ((Z . S2 bra) . Th), b2 = ((X . S1 bra) . Th) . Z (as for the gated bond)
    add(2, tc_build(zb, Z, site_tv(v2[i], OP_ID, false, cdt, "PsVSG")));
    add(2, tc_build(xb, X, site_tv(v1[i], OP_ID, false, cdt, "pmvsg")));
    add(3, tc_build(wl, zb, th));
    add(3, tc_build(wr, xb, th));
    add(4, tc_build(tr ? dense(req[i].b1, cdt, "pvmgs", {d, Du, Dl, Dd, h}) : dense(req[i].b1, cdt, "pmvsg", {d, Dl, Du, h, Dd}),
                    X, wl));
    add(4, tc_build(tr ? dense(req[i].b2, cdt, "PVsGS", {d, U, h, D, R}) : dense(req[i].b2, cdt, "PsVSG", {d, h, U, R, D}),
                    wr, Z));
    // N1 from L[c], T[c], B[c], R1; N2 from L2, T[c+1], B[c+1], R[c+2]
    for (int k = 0; k < 2; ++k) {
      const int cc = c + k;
      const int64_t xx = j.bB[cc], yy = j.bB[cc + 1], ee = j.bT[cc + 1];
      const int64_t dl = j.Dl[cc], du = j.T->leg[cc], dr = j.Dl[cc + 1], dd = j.B->leg[cc];
      TV Lk = k == 0 ? L : envv(j, L2[i], c + 1, "xlma", cdt);
      TV Tk = dense(j.T->tc[cc], cdt, "auve", {j.bT[cc], du, du, ee});
      TV Bk = dense(j.B->tc[cc], cdt, "xdgy", {xx, dd, dd, yy});
      TV Rk = k == 0 ? envv(j, R1[i], c + 1, "yrse", cdt) : envv(j, j.R[c + 2], c + 2, "yrse", cdt);
      TV y1 = tr ? dense(get(xx * du * dl * du * dl * ee), cdt, "xulvme", {xx, du, dl, du, dl, ee})
                 : dense(get(xx * dl * du * dl * du * ee), cdt, "xlumve", {xx, dl, du, dl, du, ee});
      TV y2 = tr ? dense(get(du * dl * dd * du * dl * dd * yy * ee), cdt, "uldvmgye", {du, dl, dd, du, dl, dd, yy, ee})
                 : dense(get(dl * du * dd * dl * du * dd * yy * ee), cdt, "ludmvgye", {dl, du, dd, dl, du, dd, yy, ee});
      double* out = k == 0 ? req[i].n1 : req[i].n2;
      TV n = tr ? dense(out, cdt, "uldrvmgs", {du, dl, dd, dr, du, dl, dd, dr})
                : dense(out, cdt, "lurdmvsg", {dl, du, dr, dd, dl, du, dr, dd});
      add(0, tc_build(y1, Lk, Tk));
      add(1, tc_build(y2, y1, Bk));
      add(2, tc_build(n, y2, Rk));
    }
    for (int k = 0; k < 5; ++k) rec.tc(prec, cdt, std::move(st[k]));
    for (void* p : tmp) scr.put(p);
    rec.flush(call);
  }
  // <L[k], R[k]> at k = c+1, c+2 (once per job and column)
  {
    std::vector<RedDesc> rd;
    std::vector<std::vector<char>> done(rj.size());
    for (size_t k = 0; k < rj.size(); ++k) done[k].assign(rj[k].Lc + 1, 0);
    for (size_t i = 0; i < req.size(); ++i) {
      const RJob& j = rj[jid[i]];
      for (int k = req[i].c + 1; k <= req[i].c + 2; ++k) {
        if (done[jid[i]][k]) continue;
        done[jid[i]][k] = 1;
        rd.push_back(red_desc(j.L[k], j.R[k], env_elems(j, k), j.dots + k, cdt));
      }
    }
    rec.reduce(std::move(rd));
  }
  std::vector<std::vector<double>> hd, hl, hr;
  run_and_read_dots(rec, call, rj, ctx.stream, hd, hl, hr);
  // the gated bond's scale factors of the two sites (the stored state's)
  double* s2 = (double*)call.alloc(sizeof(double) * 2 * req.size());
  std::vector<EwDesc> fill, scale;
  for (size_t i = 0; i < req.size(); ++i) {
    const size_t k = jid[i];
    const int c = req[i].c;
    const double w0 = std::sqrt(hl[k][c + 1]) * hd[k][c + 1], w1 = std::sqrt(hl[k][c + 2]) * hd[k][c + 2];
    const double sl = std::sqrt(hr[k][c + 1]) * std::fabs(w0), sr = std::sqrt(hl[k][c + 1]) * std::fabs(w1);
    if (!(std::isfinite(sl) && sl > 0.0 && std::isfinite(sr) && sr > 0.0))
      throw Error(ST_NONFINITE, "bond fit (" + std::to_string(req[i].r) + "," + std::to_string(c) +
                                    ") has a zero or non-finite scale");
    const RJob& j = rj[k];
    const int64_t d = j.s[c]->d;
    const int64_t K1 = j.Dl[c] * j.T->leg[c] * j.Dl[c + 1] * j.B->leg[c];
    const int64_t K2 = j.Dl[c + 1] * j.T->leg[c + 1] * j.Dl[c + 2] * j.B->leg[c + 1];
    for (int side = 0; side < 2; ++side) {
      EwDesc fl = ew_desc(EW_FILL, nullptr, DT_F64, s2 + 2 * i + side, DT_F64, 1);
      fl.a = side == 0 ? sl * sl : sr * sr;
      fill.push_back(fl);
      const int64_t K = side == 0 ? K1 : K2;
      double* outs[2] = {side == 0 ? req[i].n1 : req[i].n2, side == 0 ? req[i].b1 : req[i].b2};
      const int64_t ns[2] = {K * K, d * K};
      for (int t = 0; t < 2; ++t) {
        EwDesc e = ew_desc(EW_RSQRT, outs[t], DT_F64, outs[t], DT_F64, ns[t]);
        e.sptr = s2 + 2 * i + side;
        scale.push_back(e);
      }
    }
  }
  Rec rec2(&ctx, &call);
  rec2.ew(fill);
  rec2.ew(scale);
  rec2.run(call);
  dev::sync(ctx.stream);
}

}  // namespace pe
