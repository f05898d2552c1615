// Boundary-MPS environment of a finite PEPS: row absorption with ALS
// truncation (the sandwich contraction of arXiv:1311.6696, Sec. 2) and the
// row / two-row sandwiches giving norm, <S^z> and bond energies.
//
// Every routine here works on a batch of independent jobs in lockstep: each
// stage of each job becomes one descriptor, and the descriptors of all jobs
// at the same stage form one grouped launch.  Nothing here waits on the GPU
// until the whole batch has been recorded.
#include "chains.hpp"

#include <algorithm>
#include <cmath>

namespace pe {

// ---------------------------------------------------------------- Scratch ---
void* Scratch::get(size_t bytes) {
  if (bytes < 256) bytes = 256;
  for (auto it = free_.lower_bound(bytes); it != free_.end() && it->first <= 2 * bytes; ++it)
    if (!it->second.empty()) {
      void* p = it->second.back();
      it->second.pop_back();
      return p;
    }
  void* p = arena_.alloc(bytes);
  size_[p] = bytes;
  held_ += bytes;
  return p;
}

void Scratch::put(void* p) {
  if (!p) return;
  auto it = size_.find(p);
  if (it != size_.end()) free_[it->second].push_back(p);
}

namespace {

// ------------------------------------------------------ boundary planning --
// One row absorption T_out ~ T_in . row (Sec. 2): bond caps, exact product
// or ALS with QR gauge.  Frame: side 0 = rows top-down as given, side 1 =
// lattice mirrored top<->bottom (rows reversed, up/down legs swapped).
struct AJob {
  peps_env* env;
  int side, k, Lc;
  const Mps* Tin;
  Mps* Tout;
  std::vector<TV> Ak, Ab;        // row sites, labels plurd / pmvsg
  const void* lam;
  const void* rho;
  std::vector<int64_t> bin, bout, Dl, Dd;   // bonds (Lc+1), left legs (Lc+1), down legs (Lc)
  bool exact = false;
  std::vector<void*> E, F;
  std::vector<double*> X;
  std::vector<void*> Xc;
  void *P = nullptr, *Q = nullptr;
  double *N = nullptr, *W = nullptr, *R = nullptr;
  double* omega = nullptr;
  int H = 0;            // half-sweeps recorded so far
  bool conv = true;     // stopped by the tolerance (or no tolerance)
  std::vector<void*> scratch;
};

uint64_t splitmix_stream_state(uint64_t seed, uint64_t q) { return splitmix_mix(seed + (q + 1) * SPLITMIX_GAMMA); }

std::vector<int64_t> bond_caps(int64_t chi, const std::vector<int64_t>& chi_prod, const std::vector<int64_t>& Dd) {
  const int Lc = (int)Dd.size();
  const int64_t BIG = int64_t(1) << 40;
  std::vector<int64_t> full(Lc + 1, 1);
  for (int c = 0; c + 1 < Lc; ++c) {
    int64_t left = 1, right = 1;
    for (int q = 0; q <= c; ++q) left = std::min(BIG, left * Dd[q] * Dd[q]);
    for (int q = c + 1; q < Lc; ++q) right = std::min(BIG, right * Dd[q] * Dd[q]);
    full[c + 1] = std::min(std::min(chi, chi_prod[c]), std::min(left, right));
  }
  for (int c = 0; c < Lc; ++c) full[c + 1] = std::min(full[c + 1], full[c] * Dd[c] * Dd[c]);
  for (int c = Lc - 1; c >= 0; --c) full[c] = std::min(full[c], full[c + 1] * Dd[c] * Dd[c]);
  return full;
}

void cast_copies(Rec& rec, std::vector<AJob*>& js, const Opts& o, int c_only = -1) {
  if (o.cdt() == DT_F64) return;
  std::vector<EwDesc> ew;
  for (AJob* j : js)
    for (int c = 0; c < j->Lc; ++c) {
      if (c_only >= 0 && c != c_only) continue;
      ew.push_back(ew_desc(EW_COPY, j->X[c], DT_F64, j->Xc[c], DT_F32, j->bout[c] * j->Dd[c] * j->Dd[c] * j->bout[c + 1]));
    }
  rec.ew(std::move(ew));
}

TV Tview(const AJob& j, int c, const char* lbl, int cdt) {
  return dense(j.Tin->tc[c], cdt, lbl, {j.bin[c], j.Tin->leg[c], j.Tin->leg[c], j.bin[c + 1]});
}

void plan_exact(Rec& rec, Scratch& scr, std::vector<AJob*>& js, const Opts& o) {
  if (js.empty()) return;
  const int prec = o.prec(), cdt = o.cdt();
  const size_t esz = dtype_size(cdt);
  int maxLc = 0;
  for (AJob* j : js) maxLc = std::max(maxLc, j->Lc);
  // product tensors via the chain with identity environments (closings at the ends)
  for (int c = 0; c < maxLc; ++c) {
    St st(3, prec);
    std::vector<TcDesc> fin;
    std::vector<EwDesc> fills;
    std::vector<void*> tmp;
    for (AJob* j : js) {
      if (c >= j->Lc) continue;
      const int64_t Dl = j->Dl[c], Dr = j->Dl[c + 1];
      TV E, F;
      if (c == 0) {
        E = dense(j->lam, cdt, "xlma", {1, Dl, Dl, 1});
      } else {
        const int64_t nx = j->bin[c] * Dl * Dl;
        void* I = scr.get(nx * nx * esz);
        tmp.push_back(I);
        EwDesc e = ew_desc(EW_IDENTITY, nullptr, cdt, I, cdt, nx * nx);
        e.dim = (int)nx;
        e.a = 1.0;
        fills.push_back(e);
        E = dense(I, cdt, "xlma", {nx, Dl, Dl, j->bin[c]});
      }
      if (c == j->Lc - 1) {
        F = dense(j->rho, cdt, "yrse", {1, Dr, Dr, 1});
      } else {
        const int64_t ny = j->bin[c + 1] * Dr * Dr;
        void* I = scr.get(ny * ny * esz);
        tmp.push_back(I);
        EwDesc e = ew_desc(EW_IDENTITY, nullptr, cdt, I, cdt, ny * ny);
        e.dim = (int)ny;
        e.a = 1.0;
        fills.push_back(e);
        F = dense(I, cdt, "yrse", {ny, Dr, Dr, j->bin[c + 1]});
      }
      const int64_t Ee = j->bin[c + 1];
      const int64_t nP = chain_scratch_P(E.dim[0], Dl, j->Tin->leg[c], Ee, Dr, j->Dd[c]);
      // Q also holds the fused ket-bra output, which has the size of a P tensor
      const int64_t nQ = std::max(nP, E.dim[0] * j->Dd[c] * Dr * j->Ak[c].dim[0] * Dl * j->Tin->leg[c] * Ee);
      void* P = scr.get(nP * esz);
      void* Q = scr.get(nQ * esz);
      tmp.push_back(P);
      tmp.push_back(Q);
      TV y3 = chain_left(st, E, Tview(*j, c, "auve", cdt), j->Ak[c], j->Ab[c], P, Q, cdt);
      TV X = dense(j->X[c], DT_F64, "xdgy", {j->bout[c], j->Dd[c], j->Dd[c], j->bout[c + 1]});
      fin.push_back(tc_build(X, y3, F));
    }
    rec.ew(std::move(fills));
    for (size_t i = 0; i < st.s.size(); ++i) {
      rec.tc(prec, cdt, std::move(st.s[i]), false);
      rec.kb(prec, cdt, std::move(st.k[i]), false);
    }
    rec.tc(prec, DT_F64, std::move(fin), false);
    for (void* p : tmp) scr.put(p);
  }
  // left-canonical form by QR; R moves into the next tensor
  for (int c = 0; c + 1 < maxLc; ++c) {
    std::vector<QrDesc> qrs;
    std::vector<TcDesc> mv;
    for (AJob* j : js) {
      if (c + 1 >= j->Lc) continue;
      const int64_t m = j->bout[c] * j->Dd[c] * j->Dd[c], n = j->bout[c + 1];
      PE_REQUIRE(m >= n, "exact absorption: block narrower than its bond");
      qrs.push_back(qr_desc(j->X[c], n, 1, j->X[c], n, 1, j->R, n, 1, j->W, (int)m, (int)n));
      double* nx = (double*)j->env->arena.alloc(sizeof(double) * j->bout[c + 1] * j->Dd[c + 1] * j->Dd[c + 1] * j->bout[c + 2]);
      TV out = dense(nx, DT_F64, "xdgy", {n, j->Dd[c + 1], j->Dd[c + 1], j->bout[c + 2]});
      mv.push_back(tc_build(out, dense(j->R, DT_F64, "xz", {n, n}),
                            dense(j->X[c + 1], DT_F64, "zdgy", {n, j->Dd[c + 1], j->Dd[c + 1], j->bout[c + 2]})));
      j->X[c + 1] = nx;
      if (cdt == DT_F64) j->Xc[c + 1] = nx;
    }
    rec.qr(qrs);
    rec.tc(TP_F64, DT_F64, std::move(mv), false);
  }
  std::vector<RedDesc> rd;
  std::vector<EwDesc> sc;
  for (AJob* j : js) {
    const int c = j->Lc - 1;
    const int64_t n = j->bout[c] * j->Dd[c] * j->Dd[c] * j->bout[c + 1];
    rd.push_back(red_desc(j->X[c], nullptr, n, j->omega, DT_F64));
    EwDesc e = ew_desc(EW_RSQRT, j->X[c], DT_F64, j->X[c], DT_F64, n);
    e.sptr = j->omega;
    sc.push_back(e);
  }
  rec.reduce(std::move(rd));
  rec.ew(std::move(sc));
  cast_copies(rec, js, o);
}

// Views of one ALS job's tensors (contraction dtype unless noted).
struct AlsViews {
  int cdt;
  TV E(AJob* j, int c) const { return dense(j->E[c], cdt, "xlma", {j->bout[c], j->Dl[c], j->Dl[c], j->bin[c]}); }
  TV F(AJob* j, int c) const { return dense(j->F[c], cdt, "yrse", {j->bout[c], j->Dl[c], j->Dl[c], j->bin[c]}); }
  TV X(AJob* j, int c) const { return dense(j->Xc[c], cdt, "xdgy", {j->bout[c], j->Dd[c], j->Dd[c], j->bout[c + 1]}); }
  TV N(AJob* j, int c) const {   // float64 site solution
    return dense(j->N, DT_F64, "xdgy", {j->bout[c], j->Dd[c], j->Dd[c], j->bout[c + 1]});
  }
};

// ALS start: SplitMix64 tensors, right-canonical by LQ, right environments.
void als_start(Rec& rec, std::vector<AJob*>& js, const Opts& o) {
  const int prec = o.prec(), cdt = o.cdt();
  const AlsViews v{cdt};
  int maxLc = 0;
  for (AJob* j : js) maxLc = std::max(maxLc, j->Lc);
  {
    std::vector<EwDesc> f;
    for (AJob* j : js)
      for (int c = 0; c < j->Lc; ++c) {
        EwDesc e = ew_desc(EW_SPLITMIX, nullptr, DT_F64, j->X[c], DT_F64,
                           j->bout[c] * j->Dd[c] * j->Dd[c] * j->bout[c + 1]);
        const uint64_t q = (uint64_t(j->env->side0 + j->side) << 40) | (uint64_t(j->k) << 20) | uint64_t(c);
        e.key = splitmix_stream_state(j->env->opts.seed, q);
        f.push_back(e);
      }
    rec.ew(std::move(f));
  }
  for (int s = 0; s + 1 < maxLc; ++s) {
    std::vector<QrDesc> qrs;
    std::vector<TcDesc> mv;
    for (AJob* j : js) {
      const int c = j->Lc - 1 - s;
      if (c < 1) continue;
      const int64_t m = j->Dd[c] * j->Dd[c] * j->bout[c + 1], n = j->bout[c];
      qrs.push_back(qr_desc(j->X[c], 1, m, j->X[c], 1, m, j->R, n, 1, j->W, (int)m, (int)n));
      double* nx = (double*)j->env->arena.alloc(sizeof(double) * j->bout[c - 1] * j->Dd[c - 1] * j->Dd[c - 1] * n);
      TV out = dense(nx, DT_F64, "adgx", {j->bout[c - 1], j->Dd[c - 1], j->Dd[c - 1], n});
      mv.push_back(tc_build(out, dense(j->X[c - 1], DT_F64, "adgy", {j->bout[c - 1], j->Dd[c - 1], j->Dd[c - 1], n}),
                            dense(j->R, DT_F64, "xy", {n, n})));
      j->X[c - 1] = nx;
      if (cdt == DT_F64) j->Xc[c - 1] = nx;
    }
    rec.qr(qrs);
    rec.tc(TP_F64, DT_F64, std::move(mv), false);
  }
  cast_copies(rec, js, o);
  for (int s = 0; s + 1 < maxLc; ++s) {
    St st(3, prec);
    std::vector<TcDesc> env;
    for (AJob* j : js) {
      const int c = j->Lc - 1 - s;
      if (c < 1) continue;
      const double f0 = st.flops;
      TV y3 = chain_right(st, v.F(j, c + 1), Tview(*j, c, "auve", cdt), j->Ak[c], j->Ab[c], j->P, j->Q, cdt);
      env.push_back(tc_build(dense(j->F[c], cdt, "xlma", {j->bout[c], j->Dl[c], j->Dl[c], j->bin[c]}), y3, v.X(j, c)));
      j->env->flops += st.flops - f0 + tc_flops(env.back());
    }
    st.record(rec, prec, cdt);
    rec.tc(prec, cdt, std::move(env));
  }
  for (AJob* j : js) j->H = 0;
}

// Half-sweep h of every job (all at the same h): left to right for even h.
// Each site step: the local solution N = E.(T A A).F, its QR gauge, the
// environment update; the squared norm of the last N goes to omega[h].
void als_halfsweep(Rec& rec, std::vector<AJob*>& js, const Opts& o, int h) {
  const int prec = o.prec(), cdt = o.cdt();
  const AlsViews v{cdt};
  int maxLc = 0;
  for (AJob* j : js) maxLc = std::max(maxLc, j->Lc);
  const bool l2r = (h % 2 == 0);
  for (int s = 0; s < maxLc; ++s) {
    St st(3, prec);
    std::vector<TcDesc> site, env;
    std::vector<QrDesc> qrs;
    std::vector<AJob*> upd;
    for (AJob* j : js) {
      if (s >= j->Lc) continue;
      const int Lc = j->Lc;
      if (l2r) {
        const int c = s;
        const bool reuse = (h > 0 && c == 0);
        const bool need_env = c < Lc - 1;
        if (reuse && !need_env) continue;
        const double f0 = st.flops;
        TV y3 = chain_left(st, v.E(j, c), Tview(*j, c, "auve", cdt), j->Ak[c], j->Ab[c], j->P, j->Q, cdt);
        j->env->flops += st.flops - f0;
        if (!reuse) site.push_back(tc_build(v.N(j, c), y3, v.F(j, c + 1)));
        if (!reuse) j->env->flops += tc_flops(site.back());
        if (need_env) {
          const int64_t m = j->bout[c] * j->Dd[c] * j->Dd[c], n = j->bout[c + 1];
          qrs.push_back(qr_desc(j->N, n, 1, j->X[c], n, 1, nullptr, 0, 0, j->W, (int)m, (int)n));
          env.push_back(tc_build(dense(j->E[c + 1], cdt, "yrse", {j->bout[c + 1], j->Dl[c + 1], j->Dl[c + 1], j->bin[c + 1]}),
                                 y3, v.X(j, c)));
          j->env->flops += tc_flops(env.back());
          upd.push_back(j);
        }
      } else {
        const int c = Lc - 1 - s;
        const bool reuse = (c == Lc - 1);
        const bool need_env = c > 0;
        if (reuse && !need_env) continue;
        const double f0 = st.flops;
        TV y3 = chain_right(st, v.F(j, c + 1), Tview(*j, c, "auve", cdt), j->Ak[c], j->Ab[c], j->P, j->Q, cdt);
        j->env->flops += st.flops - f0;
        if (!reuse) site.push_back(tc_build(v.N(j, c), y3, v.E(j, c)));
        if (!reuse) j->env->flops += tc_flops(site.back());
        if (need_env) {
          const int64_t m = j->Dd[c] * j->Dd[c] * j->bout[c + 1], n = j->bout[c];
          qrs.push_back(qr_desc(j->N, 1, m, j->X[c], 1, m, nullptr, 0, 0, j->W, (int)m, (int)n));
          env.push_back(tc_build(dense(j->F[c], cdt, "xlma", {j->bout[c], j->Dl[c], j->Dl[c], j->bin[c]}), y3,
                                 v.X(j, c)));
          j->env->flops += tc_flops(env.back());
          upd.push_back(j);
        }
      }
    }
    st.record(rec, prec, cdt);
    rec.tc(prec, DT_F64, std::move(site));
    rec.qr(qrs);
    if (cdt != DT_F64) {
      std::vector<EwDesc> ew;
      for (AJob* j : upd) {
        const int c = l2r ? s : j->Lc - 1 - s;
        ew.push_back(ew_desc(EW_COPY, j->X[c], DT_F64, j->Xc[c], DT_F32,
                             j->bout[c] * j->Dd[c] * j->Dd[c] * j->bout[c + 1]));
      }
      rec.ew(std::move(ew));
    }
    rec.tc(prec, cdt, std::move(env));
  }
  std::vector<RedDesc> rd;
  for (AJob* j : js) {
    const int c = l2r ? j->Lc - 1 : 0;
    rd.push_back(red_desc(j->N, nullptr, j->bout[c] * j->Dd[c] * j->Dd[c] * j->bout[c + 1], j->omega + h, DT_F64));
    j->H = h + 1;
  }
  rec.reduce(std::move(rd));
}

// Normalise each job's centre tensor (site Lc-1 after an odd number of
// half-sweeps, site 0 after an even one) and refresh the compute-dtype copies.
void als_finish(Rec& rec, std::vector<AJob*>& js, const Opts& o) {
  std::vector<EwDesc> sc;
  for (AJob* j : js) {
    const int c = (j->H % 2 == 1) ? j->Lc - 1 : 0;
    EwDesc e = ew_desc(EW_RSQRT, j->N, DT_F64, j->X[c], DT_F64, j->bout[c] * j->Dd[c] * j->Dd[c] * j->bout[c + 1]);
    e.sptr = j->omega + (j->H - 1);
    sc.push_back(e);
  }
  rec.ew(std::move(sc));
  cast_copies(rec, js, o);
}

// ALS truncation of every job of one precision: `o.halfsweeps` half-sweeps,
// then, for jobs with a tolerance, one more at a time (each decided on the
// host after the GPU has caught up) until |omega_h - omega_(h-1)| <=
// tol * omega_h or the job's cap.
void plan_als(Rec& rec, Arena& call, Ctx& ctx, std::vector<AJob*>& js, const Opts& o) {
  if (js.empty()) return;
  als_start(rec, js, o);
  for (int h = 0; h < o.halfsweeps; ++h) als_halfsweep(rec, js, o, h);
  std::vector<AJob*> act;
  for (AJob* j : js) {
    j->conv = true;
    if (j->env->opts.tol > 0.0 && j->env->opts.max_halfsweeps > j->H) act.push_back(j);
  }
  std::vector<double> w(2 * js.size());
  while (!act.empty()) {
    Gather g;
    for (AJob* j : act) g.add(j->omega + (j->H - 2), 2);
    g.record(rec, call);
    rec.flush(call);
    g.read(ctx.stream);
    std::copy(g.host.begin(), g.host.end(), w.begin());
    std::vector<AJob*> next;
    for (size_t i = 0; i < act.size(); ++i) {
      AJob* j = act[i];
      const double a = w[2 * i], b = w[2 * i + 1];
      if (!(std::isfinite(a) && std::isfinite(b) && b > 0.0))
        throw Error(ST_NONFINITE, "boundary row " + std::to_string(j->k) + " has squared norm " + std::to_string(b));
      if (std::fabs(b - a) <= j->env->opts.tol * b) continue;
      if (j->H >= j->env->opts.max_halfsweeps) {
        j->conv = false;
        continue;
      }
      next.push_back(j);
    }
    if (next.empty()) break;
    als_halfsweep(rec, next, o, next[0]->H);
    act.swap(next);
  }
  als_finish(rec, js, o);
}

}  // namespace

// Frame helpers: side 0 is the lattice as given, side 1 its top<->bottom mirror.
static const Site& frame_site(const Lattice& L, int side, int k, int c) {
  return side == 0 ? L.at(k, c) : L.at(L.Lr - 1 - k, c);
}

static Mps closing_mps(const Lattice& L, int side) {
  Mps m;
  m.bond.assign(L.Lc + 1, 1);
  for (int c = 0; c < L.Lc; ++c) {
    const Site& s = frame_site(L, side, 0, c);
    m.leg.push_back(side == 0 ? s.Du : s.Dd);
    m.tc.push_back(side == 0 ? L.tau[c] : L.beta[c]);
    m.t64.push_back(nullptr);
  }
  return m;
}

void plan_boundaries(Ctx& ctx, std::vector<peps_env*>& envs) {
  Arena call(&ctx.pool);
  Rec rec(&ctx, &call);
  Scratch scr(call);
  int maxLr = 0;
  for (peps_env* e : envs) {
    const Lattice& L = e->lat;
    e->top.clear();
    e->bot.clear();
    e->top.push_back(closing_mps(L, 0));
    e->bot.push_back(closing_mps(L, 1));
    e->top.reserve(L.Lr);
    e->bot.reserve(L.Lr);
    maxLr = std::max(maxLr, L.Lr);
  }
  for (int k = 0; k + 1 < maxLr; ++k) {
    std::vector<AJob> jobs;
    for (peps_env* e : envs) {
      const Lattice& L = e->lat;
      if (k + 1 >= L.Lr) continue;
      for (int side = 0; side < 2; ++side) {
        std::vector<Mps>& vec = side == 0 ? e->top : e->bot;
        vec.emplace_back();
        AJob j;
        j.env = e;
        j.side = side;
        j.k = k;
        j.Lc = L.Lc;
        j.Tin = &vec[k];
        j.Tout = &vec[k + 1];
        const int cdt = e->opts.cdt();
        const int orow = side == 0 ? k : L.Lr - 1 - k;
        j.lam = L.lam[orow];
        j.rho = L.rho[orow];
        j.bin = std::vector<int64_t>(j.Tin->bond.begin(), j.Tin->bond.end());
        for (int c = 0; c < L.Lc; ++c) {
          const Site& s = frame_site(L, side, k, c);
          j.Ak.push_back(site_tv(s, OP_ID, side == 1, cdt, "plurd"));
          j.Ab.push_back(site_tv(s, OP_ID, side == 1, cdt, "pmvsg"));
          j.Dl.push_back(s.Dl);
          j.Dd.push_back(side == 0 ? s.Dd : s.Du);
          PE_REQUIRE((side == 0 ? s.Du : s.Dd) == j.Tin->leg[c], "boundary leg mismatch");
        }
        j.Dl.push_back(frame_site(L, side, k, L.Lc - 1).Dr);
        std::vector<int64_t> prodb(L.Lc > 1 ? L.Lc - 1 : 0);
        for (int c = 0; c + 1 < L.Lc; ++c) prodb[c] = j.bin[c + 1] * j.Dl[c + 1] * j.Dl[c + 1];
        j.bout = bond_caps(e->opts.chi, prodb, j.Dd);
        j.exact = true;
        for (int c = 0; c + 1 < L.Lc; ++c) j.exact = j.exact && (j.bout[c + 1] == prodb[c]);
        jobs.push_back(std::move(j));
      }
    }
    // allocate outputs and scratch
    std::vector<AJob*> ex, als;
    for (AJob& j : jobs) {
      peps_env* e = j.env;
      const int cdt = e->opts.cdt();
      const size_t esz = dtype_size(cdt);
      const int H = j.exact ? 1 : std::max(e->opts.halfsweeps, e->opts.max_halfsweeps);
      j.omega = (double*)e->arena.alloc(sizeof(double) * H);
      int64_t maxX = 1, maxQR = 1, maxR = 1, maxP = 1, maxQ = 1;
      for (int c = 0; c < j.Lc; ++c) {
        const int64_t nx = j.bout[c] * j.Dd[c] * j.Dd[c] * j.bout[c + 1];
        maxX = std::max(maxX, nx);
        maxQR = std::max(maxQR, nx * std::max(j.bout[c], j.bout[c + 1]));
        maxR = std::max(maxR, std::max(j.bout[c], j.bout[c + 1]));
        j.X.push_back((double*)e->arena.alloc(sizeof(double) * nx));
        j.Xc.push_back(cdt == DT_F64 ? (void*)j.X.back() : e->arena.alloc(esz * nx));
        const int64_t Dl = j.Dl[c], Dr = j.Dl[c + 1], Du = j.Tin->leg[c], Dd = j.Dd[c];
        const int64_t xo = std::max(j.bout[c], j.bout[c + 1]);
        const int64_t ain = std::max(j.bin[c], j.bin[c + 1]);
        maxP = std::max(maxP, xo * ain * std::max(Dl, Dr) * std::max(Dl, Dr) * std::max(Du, Dd) * std::max(Du, Dd));
        maxQ = std::max(maxQ, xo * ain * std::max(Dl, Dr) * std::max(Dl, Dr) * std::max(Du, Dd) * std::max(Du, Dd) *
                                  j.Ak[c].dim[0]);
      }
      j.W = (double*)scr.get(sizeof(double) * 2 * maxQR);
      j.R = (double*)scr.get(sizeof(double) * maxR * maxR);
      j.scratch = {j.W, j.R};
      if (!j.exact) {
        j.N = (double*)scr.get(sizeof(double) * maxX);
        j.P = scr.get(esz * maxP);
        j.Q = scr.get(esz * maxQ);
        j.scratch.insert(j.scratch.end(), {j.N, j.P, j.Q});
        j.E.assign(j.Lc + 1, nullptr);
        j.F.assign(j.Lc + 1, nullptr);
        j.E[0] = const_cast<void*>(j.lam);
        j.F[j.Lc] = const_cast<void*>(j.rho);
        for (int c = 1; c < j.Lc; ++c) {
          const int64_t n = j.bout[c] * j.Dl[c] * j.Dl[c] * j.bin[c];
          j.E[c] = scr.get(esz * n);
          j.F[c] = scr.get(esz * n);
          j.scratch.push_back(j.E[c]);
          j.scratch.push_back(j.F[c]);
        }
        als.push_back(&j);
      } else {
        ex.push_back(&j);
      }
    }
    // one grouped chain per (precision, half-sweep count); seeds are per job
    std::vector<std::pair<int, int>> groups;
    for (AJob& j : jobs) {
      const std::pair<int, int> g{j.env->opts.dtype, j.env->opts.halfsweeps};
      if (std::find(groups.begin(), groups.end(), g) == groups.end()) groups.push_back(g);
    }
    std::sort(groups.begin(), groups.end());
    for (const auto& g : groups) {
      std::vector<AJob*> a, b;
      for (AJob* j : ex)
        if (j->env->opts.dtype == g.first && j->env->opts.halfsweeps == g.second) a.push_back(j);
      for (AJob* j : als)
        if (j->env->opts.dtype == g.first && j->env->opts.halfsweeps == g.second) b.push_back(j);
      if (a.empty() && b.empty()) continue;
      const Opts& o = (a.empty() ? b[0] : a[0])->env->opts;
      plan_exact(rec, scr, a, o);
      plan_als(rec, call, ctx, b, o);
    }
    for (AJob& j : jobs) {
      j.Tout->t64 = j.X;
      j.Tout->tc.assign(j.Xc.begin(), j.Xc.end());
      j.Tout->bond.assign(j.bout.begin(), j.bout.end());
      j.Tout->leg.assign(j.Dd.begin(), j.Dd.end());
      j.Tout->omega = j.omega;
      j.Tout->n_omega = j.exact ? 1 : j.H;
      j.Tout->truncated = !j.exact;
      j.Tout->converged = j.exact || j.conv;
      for (void* p : j.scratch) scr.put(p);
    }
    rec.flush(call);   // the GPU starts on this row while the next one is planned
  }
  // log-scales: the FP64 sums of log(omega)/2 over the absorbed rows of every
  // side run on the device; one copy brings all of them back
  std::vector<EwDesc> acc;
  size_t nlog = 0;
  for (peps_env* e : envs) nlog += 2 * (size_t)e->lat.Lr;
  double* logs = (double*)call.alloc(sizeof(double) * std::max<size_t>(nlog, 1));
  // every side's list of omega pointers in one device copy
  std::vector<const double*> w;
  std::vector<size_t> first;
  size_t at = 0;
  for (peps_env* e : envs) {
    for (int side = 0; side < 2; ++side) {
      std::vector<Mps>& vec = side == 0 ? e->top : e->bot;
      first.push_back(w.size());
      for (size_t k = 1; k < vec.size(); ++k) w.push_back(vec[k].omega + (vec[k].n_omega - 1));
      EwDesc d = ew_desc(EW_LOGACC, nullptr, DT_F64, logs + at, DT_F64, (int64_t)(w.size() - first.back()));
      acc.push_back(d);
      at += e->lat.Lr;
    }
  }
  if (!w.empty()) {
    const double** wd = (const double**)rec.aux(call, w.data(), w.size() * sizeof(const double*));
    for (size_t i = 0; i < acc.size(); ++i)
      if (acc[i].n) acc[i].src = wd + first[i];
  }
  rec.ew(std::move(acc));
  rec.run(call);
  std::vector<double> hl(std::max<size_t>(nlog, 1));
  dev::d2h(hl.data(), logs, sizeof(double) * nlog, ctx.stream);
  dev::sync(ctx.stream);
  at = 0;
  for (peps_env* e : envs) {
    const int Lr = e->lat.Lr;
    for (int side = 0; side < 2; ++side) {
      std::vector<double>& lg = side == 0 ? e->top_log : e->bot_log;
      lg.assign(hl.begin() + at, hl.begin() + at + Lr);
      at += Lr;
      for (int k = 1; k < Lr; ++k)
        if (!std::isfinite(lg[k]))
          throw Error(ST_NONFINITE, "boundary row " + std::to_string(k - 1) + " (side " + std::to_string(side) +
                                        ") has a non-finite or non-positive squared norm");
      if (e->opts.strict) {
        const std::vector<Mps>& vec = side == 0 ? e->top : e->bot;
        for (size_t k = 1; k < vec.size(); ++k)
          if (!vec[k].converged)
            throw Error(ST_NOT_CONVERGED, "boundary row " + std::to_string(k - 1) + " (side " + std::to_string(side) +
                                              ") reached max_halfsweeps before the tolerance");
      }
    }
  }
}

}  // namespace pe
