// extern "C" entry points of libpepsenv (declared in include/peps_env.h).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <functional>

#include "../../include/peps_env.h"
#include "planner.hpp"
#include "chains.hpp"

namespace pe {
void* noalloc_scratch(int device);   // noalloc.hip
namespace {

thread_local std::string g_err;

peps_status fail(int code, const std::string& msg) {
  g_err = msg;
  return (peps_status)code;
}

template <class F>
peps_status guarded(F&& f) {
  try {
    g_err.clear();
    f();
    return PEPS_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(ST_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(ST_INVALID, e.what());
  }
}

// spin-1/2 operators on the ket physical leg (index 0 = up)
const double OPS[4][4] = {
    {1.0, 0.0, 0.0, 1.0},     // identity
    {0.5, 0.0, 0.0, -0.5},    // S^z
    {0.0, 1.0, 0.0, 0.0},     // S^+
    {0.0, 0.0, 1.0, 0.0},     // S^-
};

void validate_state(const peps_state& s, int idx) {
  const std::string w = "state " + std::to_string(idx) + ": ";
  PE_REQUIRE(s.rows >= 1 && s.cols >= 1, w + "rows and cols must be >= 1");
  PE_REQUIRE(s.dims && s.site, w + "dims and site must not be NULL");
  if (s.phys != 2) throw Error(ST_UNSUPPORTED, w + "the spin-1/2 observables need phys == 2");
  for (int r = 0; r < s.rows; ++r)
    for (int c = 0; c < s.cols; ++c) {
      const int32_t* d = s.dims + 5 * ((size_t)r * s.cols + c);
      const std::string at = w + "site (" + std::to_string(r) + "," + std::to_string(c) + ") ";
      for (int k = 0; k < 5; ++k) PE_REQUIRE(d[k] >= 1 && d[k] <= 4096, at + "has a dimension outside [1, 4096]");
      PE_REQUIRE(d[0] == s.phys, at + "physical dimension differs from phys");
      PE_REQUIRE(s.site[(size_t)r * s.cols + c] != nullptr, at + "has a NULL tensor");
      if (c == 0) PE_REQUIRE(d[1] == 1, at + "left edge leg must have dimension 1");
      if (c == s.cols - 1) PE_REQUIRE(d[3] == 1, at + "right edge leg must have dimension 1");
      if (r == 0) PE_REQUIRE(d[2] == 1, at + "top edge leg must have dimension 1");
      if (r == s.rows - 1) PE_REQUIRE(d[4] == 1, at + "bottom edge leg must have dimension 1");
      if (c + 1 < s.cols) PE_REQUIRE(d[3] == (d + 5)[1], at + "right leg does not match its neighbour");
      if (r + 1 < s.rows) PE_REQUIRE(d[4] == (d + 5 * s.cols)[2], at + "down leg does not match its neighbour");
    }
}

Opts make_opts(const peps_env_opts* o, int32_t allowed_flags = 0) {
  PE_REQUIRE(o != nullptr, "opts must not be NULL");
  PE_REQUIRE(o->chi >= 1, "chi must be >= 1");
  PE_REQUIRE(o->dtype >= PEPS_F64 && o->dtype <= PEPS_BF16, "unknown dtype");
  PE_REQUIRE(o->halfsweeps >= 0 && o->halfsweeps <= 256, "halfsweeps must be in [0, 256]");
  PE_REQUIRE((o->flags & ~(allowed_flags | PEPS_OPTS_STRICT)) == 0, "unsupported flags");
  PE_REQUIRE(o->reserved == 0, "reserved must be 0");
  PE_REQUIRE(std::isfinite(o->tol) && o->tol >= 0.0 && o->tol < 1.0, "tol must be in [0, 1)");
  Opts r;
  r.chi = o->chi;
  r.dtype = o->dtype;
  r.halfsweeps = o->halfsweeps == 0 ? 4 : o->halfsweeps;
  r.seed = o->seed;
  r.columns = (o->flags & PEPS_OPTS_COLUMNS) != 0;
  r.strict = (o->flags & PEPS_OPTS_STRICT) != 0;
  r.tol = o->tol;
  if (r.tol > 0.0) {
    r.halfsweeps = std::max(r.halfsweeps, 2);
    const int cap = o->max_halfsweeps == 0 ? std::max(40, r.halfsweeps) : o->max_halfsweeps;
    PE_REQUIRE(cap >= r.halfsweeps && cap <= 256, "max_halfsweeps must be in [halfsweeps, 256]");
    r.max_halfsweeps = cap;
  } else {
    PE_REQUIRE(o->max_halfsweeps == 0 || o->max_halfsweeps >= r.halfsweeps,
               "max_halfsweeps must be 0 or >= halfsweeps");
    r.max_halfsweeps = r.halfsweeps;
  }
  return r;
}

// Read-only pass over every input tensor of the used states: fails with
// NONFINITE, naming a site, if any entry is NaN or Inf.  Nothing is written
// but one flag in scratch memory.
void check_finite(Ctx& C, const peps_state* st, int n_states, const std::vector<char>* used = nullptr) {
  Arena tmp(&C.pool);
  Rec rec(&C);
  double* flag = (double*)tmp.alloc(sizeof(double));
  std::vector<EwDesc> clear{ew_desc(EW_FILL, nullptr, DT_F64, flag, DT_F64, 1)};
  std::vector<EwDesc> chk;
  std::vector<std::pair<int, int>> who;
  for (int i = 0; i < n_states; ++i) {
    if (used && !(*used)[i]) continue;
    for (int k = 0; k < st[i].rows * st[i].cols; ++k) {
      const int32_t* d = st[i].dims + 5 * k;
      const int64_t n = (int64_t)d[0] * d[1] * d[2] * d[3] * d[4];
      EwDesc e = ew_desc(EW_NONFINITE, st[i].site[k], DT_F64, flag, DT_F64, n);
      e.a = (double)(who.size() + 1);
      who.push_back({i, k});
      chk.push_back(e);
    }
  }
  rec.ew(std::move(clear));
  rec.ew(std::move(chk));
  rec.run(tmp);
  double f = 0.0;
  dev::d2h(&f, flag, sizeof(double), C.stream);
  dev::sync(C.stream);
  if (f != 0.0) {
    const auto& w = who[(size_t)f - 1];
    const int cols = st[w.first].cols;
    throw Error(ST_NONFINITE, "state " + std::to_string(w.first) + ": site (" + std::to_string(w.second / cols) + "," +
                                  std::to_string(w.second % cols) + ") has a NaN or Inf entry");
  }
}

// Packs the caller's float64 sites into `owner`'s arena: identity, S^z, S^+,
// S^- applied to the ket leg, in the contraction dtype.
struct Packed {
  std::vector<std::unique_ptr<Site>> sites;
};

void pack_state(Rec& rec, Arena& arena, const peps_state& s, int cdt, std::vector<std::unique_ptr<Site>>& out) {
  std::vector<EwDesc> ew;
  const size_t esz = dtype_size(cdt);
  for (int i = 0; i < s.rows * s.cols; ++i) {
    const int32_t* d = s.dims + 5 * i;
    auto st = std::make_unique<Site>();
    st->d = d[0];
    st->Dl = d[1];
    st->Du = d[2];
    st->Dr = d[3];
    st->Dd = d[4];
    const int64_t n = (int64_t)d[0] * d[1] * d[2] * d[3] * d[4];
    for (int op = 0; op < 4; ++op) {
      st->op[op] = arena.alloc(esz * n);
      EwDesc e = ew_desc(op == 0 ? EW_COPY : EW_PHYS, s.site[i], DT_F64, st->op[op], cdt, n);
      for (int k = 0; k < 4; ++k) e.op[k] = OPS[op][k];
      ew.push_back(e);
    }
    out.push_back(std::move(st));
  }
  rec.ew(std::move(ew));
}

// The transposed lattice of `e` (rows <-> columns, left/right legs <-> up/down
// legs) as an environment whose sites are views of e's packed buffers: its
// top and bottom boundaries are e's left and right ones.
std::unique_ptr<peps_env> transposed_env(const peps_env& e) {
  auto t = std::make_unique<peps_env>(e.ctxref);
  t->opts = e.opts;
  t->opts.columns = false;
  t->side0 = 2;
  const Lattice& L = e.lat;
  Lattice& T = t->lat;
  T.Lr = L.Lc;
  T.Lc = L.Lr;
  for (int c = 0; c < L.Lc; ++c)
    for (int r = 0; r < L.Lr; ++r) {
      const Site& s = L.at(r, c);
      PE_REQUIRE(!s.tr, "a transposed lattice is not transposed again");
      auto v = std::make_unique<Site>(s);
      v->Dl = s.Du;
      v->Du = s.Dl;
      v->Dr = s.Dd;
      v->Dd = s.Dr;
      v->tr = true;
      T.s.push_back(v.get());
      t->sites.push_back(std::move(v));
    }
  T.lam = L.tau;
  T.rho = L.beta;
  T.tau = L.lam;
  T.beta = L.rho;
  return t;
}

void* make_one(Rec& rec, Arena& arena, int cdt) {
  void* p = arena.alloc(16);
  std::vector<EwDesc> ew{ew_desc(EW_FILL, nullptr, cdt, p, cdt, 1)};
  ew[0].a = 1.0;
  rec.ew(std::move(ew));
  return p;
}

}  // namespace

void validate_state_public(const peps_state& s, int idx) { validate_state(s, idx); }
void check_finite_public(Ctx& C, const peps_state* st, int n_states, const std::vector<char>& used) {
  check_finite(C, st, n_states, &used);
}
Opts make_opts_public(const peps_env_opts* o) { return make_opts(o, PEPS_OPTS_COLUMNS); }
std::unique_ptr<peps_env> transposed_env_public(const peps_env& e) { return transposed_env(e); }
void pack_state_public(Rec& rec, Arena& arena, const peps_state& s, int cdt, std::vector<std::unique_ptr<Site>>& out) {
  pack_state(rec, arena, s, cdt, out);
}
void* make_one_public(Rec& rec, Arena& arena, int cdt) { return make_one(rec, arena, cdt); }
peps_status guarded_public(const std::function<void()>& f) { return guarded(f); }

}  // namespace pe

using namespace pe;

extern "C" {

const char* peps_last_error(void) { return g_err.c_str(); }

peps_status peps_ctx_create(int32_t device, void* hip_stream, peps_ctx** out) {
  return guarded([&] {
    PE_REQUIRE(out != nullptr, "out must not be NULL");
    *out = nullptr;
    const int n = dev::device_count();
    PE_REQUIRE(device >= 0 && device < n, "no such HIP device");
    dev::set_device(device);
    noalloc_scratch(device);   // the fixed QR workspace's device address, once per device
    std::unique_ptr<peps_ctx> c(new peps_ctx());
    c->c = std::make_shared<Ctx>();
    c->c->device = device;
    c->c->stream = (hipStream_t)hip_stream;
    *out = c.release();
  });
}

void peps_ctx_destroy(peps_ctx* ctx) {
  if (!ctx) return;
  try {
    dev::sync(ctx->c->stream);
  } catch (...) {
  }
  delete ctx;
}

peps_status peps_env_boundary(peps_ctx* ctx, const peps_state* st, int32_t n_states, const peps_env_opts* opts,
                              peps_env** out) {
  std::vector<peps_env*> made;
  peps_status s = guarded([&] {
    PE_REQUIRE(ctx && st && out, "ctx, st and out must not be NULL");
    PE_REQUIRE(n_states >= 1, "n_states must be >= 1");
    PE_REQUIRE(opts != nullptr, "opts must not be NULL");
    const bool per_state = (opts->flags & PEPS_OPTS_PER_STATE) != 0;
    std::vector<Opts> os;
    for (int i = 0; i < n_states; ++i) {
      const peps_env_opts* oi = per_state ? opts + i : opts;
      PE_REQUIRE(!per_state || (oi->flags & PEPS_OPTS_PER_STATE), "every per-state options record carries the flag");
      os.push_back(make_opts(oi, PEPS_OPTS_PER_STATE | PEPS_OPTS_COLUMNS));
    }
    for (int i = 0; i < n_states; ++i) validate_state(st[i], i);
    dev::set_device(ctx->c->device);
    check_finite(*ctx->c, st, n_states);
    Arena tmp(&ctx->c->pool);
    Rec rec(ctx->c.get());
    for (int i = 0; i < n_states; ++i) {
      const Opts& o = os[i];
      auto* e = new peps_env(ctx->c);
      made.push_back(e);
      e->opts = o;
      pack_state(rec, e->arena, st[i], o.cdt(), e->sites);
      void* one = make_one(rec, e->arena, o.cdt());
      Lattice& L = e->lat;
      L.Lr = st[i].rows;
      L.Lc = st[i].cols;
      for (auto& p : e->sites) L.s.push_back(p.get());
      L.lam.assign(L.Lr, one);
      L.rho.assign(L.Lr, one);
      L.tau.assign(L.Lc, one);
      L.beta.assign(L.Lc, one);
      if (o.columns) e->col = transposed_env(*e);
    }
    rec.run(tmp);
    std::vector<peps_env*> all(made);
    for (peps_env* e : made)
      if (e->col) all.push_back(e->col.get());
    plan_boundaries(*ctx->c, all);   // row and column boundaries in one batched run
    for (int i = 0; i < n_states; ++i) out[i] = made[i];
  });
  if (s != PEPS_OK) {
    for (peps_env* e : made) delete e;
    if (out && n_states > 0)
      for (int i = 0; i < n_states; ++i) out[i] = nullptr;
  }
  return s;
}

peps_status peps_expect(peps_ctx* ctx, peps_env* const* env, int32_t n_env, peps_result* out) {
  return guarded([&] {
    PE_REQUIRE(ctx && env && out, "ctx, env and out must not be NULL");
    PE_REQUIRE(n_env >= 1, "n_env must be >= 1");
    std::vector<peps_env*> es;
    for (int i = 0; i < n_env; ++i) {
      PE_REQUIRE(env[i] != nullptr, "NULL environment");
      PE_REQUIRE(env[i]->ctx == ctx->c.get(), "environment belongs to another context");
      PE_REQUIRE(out[i].sz && out[i].bond, "result buffers must not be NULL");
      es.push_back(env[i]);
    }
    dev::set_device(ctx->c->device);
    std::vector<double> f0, f1;
    for (peps_env* e : es) {
      f0.push_back(e->flops);
      f1.push_back(e->col ? e->col->flops : 0.0);
    }
    std::vector<ExpectOut> res;
    plan_expect(*ctx->c, es, res);
    for (int i = 0; i < n_env; ++i) {
      const ExpectOut& r = res[i];
      for (double v : r.sz)
        if (!std::isfinite(v) && !es[i]->window) throw Error(ST_NONFINITE, "non-finite <S^z>");
      out[i].log_norm = r.log_norm;
      out[i].norm_sign = r.sign;
      std::memcpy(out[i].sz, r.sz.data(), sizeof(double) * r.sz.size());
      std::memcpy(out[i].bond, r.bond.data(), sizeof(double) * r.bond.size());
      out[i].flops = es[i]->flops + (es[i]->col ? es[i]->col->flops : 0.0);
      es[i]->flops = f0[i];   // boundary flops stay; this call's sandwich flops are reported once
      if (es[i]->col) es[i]->col->flops = f1[i];
    }
  });
}

void peps_env_free(peps_env* env) { delete env; }

peps_status peps_bond_env(peps_ctx* ctx, const peps_bond_req* req, int32_t n_req, double* flops) {
  return guarded([&] {
    PE_REQUIRE(ctx && req, "ctx and req must not be NULL");
    PE_REQUIRE(n_req >= 1, "n_req must be >= 1");
    std::vector<BondReq> rs;
    for (int i = 0; i < n_req; ++i) {
      const peps_bond_req& q = req[i];
      const std::string w = "request " + std::to_string(i) + ": ";
      PE_REQUIRE(q.env != nullptr && q.gate != nullptr, w + "env and gate must not be NULL");
      PE_REQUIRE(q.b_left != nullptr || q.b_right != nullptr, w + "no output requested");
      PE_REQUIRE(q.env->ctx == ctx->c.get(), w + "environment belongs to another context");
      PE_REQUIRE(q.dir == 0 || q.dir == 1, w + "dir must be 0 or 1");
      if (q.dir == 0) {
        PE_REQUIRE(q.r >= 0 && q.r < q.env->lat.Lr && q.c >= 0 && q.c + 1 < q.env->lat.Lc,
                   w + "bond outside the lattice");
        rs.push_back(BondReq{q.env, q.r, q.c, q.gate, q.b_left, q.b_right, false});
      } else {
        PE_REQUIRE(q.env->col != nullptr, w + "dir 1 needs an environment built with PEPS_OPTS_COLUMNS");
        PE_REQUIRE(q.r >= 0 && q.r + 1 < q.env->lat.Lr && q.c >= 0 && q.c < q.env->lat.Lc,
                   w + "bond outside the lattice");
        // row c of the transposed lattice, bond (r, r+1) along it
        rs.push_back(BondReq{q.env->col.get(), q.c, q.r, q.gate, q.b_left, q.b_right, true});
      }
    }
    dev::set_device(ctx->c->device);
    std::vector<peps_env*> es;
    std::vector<double> f0;
    for (const BondReq& q : rs)
      if (std::find(es.begin(), es.end(), q.e) == es.end()) {
        es.push_back(q.e);
        f0.push_back(q.e->flops);
      }
    double fl = 0.0;
    try {
      plan_bond_env(*ctx->c, rs, fl);
    } catch (...) {
      for (size_t k = 0; k < es.size(); ++k) es[k]->flops = f0[k];
      throw;
    }
    for (size_t k = 0; k < es.size(); ++k) {
      fl += es[k]->flops - f0[k];
      es[k]->flops = f0[k];
    }
    if (flops) *flops = fl;
  });
}

peps_status peps_bond_fit(peps_ctx* ctx, const peps_fit_req* req, int32_t n_req, double* flops) {
  return guarded([&] {
    PE_REQUIRE(ctx && req, "ctx and req must not be NULL");
    PE_REQUIRE(n_req >= 1, "n_req must be >= 1");
    std::vector<FitReq> rs;
    for (int i = 0; i < n_req; ++i) {
      const peps_fit_req& q = req[i];
      const std::string w = "request " + std::to_string(i) + ": ";
      PE_REQUIRE(q.env && q.gate && q.s1 && q.s2, w + "env, gate, s1 and s2 must not be NULL");
      PE_REQUIRE(q.n1 && q.b1 && q.n2 && q.b2, w + "n1, b1, n2 and b2 must not be NULL");
      PE_REQUIRE(q.env->ctx == ctx->c.get(), w + "environment belongs to another context");
      PE_REQUIRE(q.dir == 0 || q.dir == 1, w + "dir must be 0 or 1");
      FitReq f{q.env, q.r, q.c, q.gate, q.s1, q.s2, q.n1, q.b1, q.n2, q.b2, false};
      if (q.dir == 0) {
        PE_REQUIRE(q.r >= 0 && q.r < q.env->lat.Lr && q.c >= 0 && q.c + 1 < q.env->lat.Lc,
                   w + "bond outside the lattice");
      } else {
        PE_REQUIRE(q.env->col != nullptr, w + "dir 1 needs an environment built with PEPS_OPTS_COLUMNS");
        PE_REQUIRE(q.r >= 0 && q.r + 1 < q.env->lat.Lr && q.c >= 0 && q.c < q.env->lat.Lc,
                   w + "bond outside the lattice");
        f.e = q.env->col.get();
        f.r = q.c;
        f.c = q.r;
        f.tr = true;
      }
      rs.push_back(f);
    }
    dev::set_device(ctx->c->device);
    std::vector<peps_env*> es;
    std::vector<double> f0;
    for (const FitReq& q : rs)
      if (std::find(es.begin(), es.end(), q.e) == es.end()) {
        es.push_back(q.e);
        f0.push_back(q.e->flops);
      }
    double fl = 0.0;
    try {
      plan_bond_fit(*ctx->c, rs, fl);
    } catch (...) {
      for (size_t k = 0; k < es.size(); ++k) es[k]->flops = f0[k];
      throw;
    }
    for (size_t k = 0; k < es.size(); ++k) {
      fl += es[k]->flops - f0[k];
      es[k]->flops = f0[k];
    }
    if (flops) *flops = fl;
  });
}

peps_status peps_boundary_overlap(peps_ctx* ctx, peps_overlap_req* req, int32_t n_req) {
  return guarded([&] {
    PE_REQUIRE(ctx && req, "ctx and req must not be NULL");
    PE_REQUIRE(n_req >= 1, "n_req must be >= 1");
    std::vector<OvReq> rs;
    for (int i = 0; i < n_req; ++i) {
      const peps_overlap_req& q = req[i];
      const std::string w = "request " + std::to_string(i) + ": ";
      PE_REQUIRE(q.env_a && q.env_b, w + "environments must not be NULL");
      PE_REQUIRE(q.env_a->ctx == ctx->c.get() && q.env_b->ctx == ctx->c.get(), w + "environment of another context");
      PE_REQUIRE(q.side >= 0 && q.side <= 3, w + "side must be 0..3");
      const Mps* m[2];
      for (int t = 0; t < 2; ++t) {
        peps_env* e = t == 0 ? q.env_a : q.env_b;
        if (q.side >= 2) {
          PE_REQUIRE(e->col != nullptr, w + "sides 2 and 3 need an environment built with PEPS_OPTS_COLUMNS");
          e = e->col.get();
        }
        const std::vector<Mps>& v = (q.side & 1) == 0 ? e->top : e->bot;
        PE_REQUIRE(q.k >= 1 && q.k < (int)v.size(), w + "k must be in [1, rows)");
        m[t] = &v[q.k];
      }
      PE_REQUIRE(m[0]->leg == m[1]->leg, w + "boundaries of different lattices");
      rs.push_back(OvReq{m[0], m[1], {0.0, 0.0, 0.0}});
    }
    dev::set_device(ctx->c->device);
    plan_overlap(*ctx->c, rs);
    for (int i = 0; i < n_req; ++i) {
      req[i].xy = rs[i].out[0];
      req[i].xx = rs[i].out[1];
      req[i].yy = rs[i].out[2];
    }
  });
}

peps_status peps_site_env(peps_ctx* ctx, peps_site_req* req, int32_t n_req, double* flops) {
  return guarded([&] {
    PE_REQUIRE(ctx && req, "ctx and req must not be NULL");
    PE_REQUIRE(n_req >= 1, "n_req must be >= 1");
    std::vector<SiteReq> rs;
    for (int i = 0; i < n_req; ++i) {
      const peps_site_req& q = req[i];
      const std::string w = "request " + std::to_string(i) + ": ";
      PE_REQUIRE(q.env != nullptr && q.n != nullptr, w + "env and n must not be NULL");
      PE_REQUIRE(q.env->ctx == ctx->c.get(), w + "environment belongs to another context");
      PE_REQUIRE(q.r >= 0 && q.r < q.env->lat.Lr && q.c >= 0 && q.c < q.env->lat.Lc, w + "site outside the lattice");
      PE_REQUIRE(q.dir == 0 || q.dir == 1, w + "dir must be 0 or 1");
      if (q.dir == 0) {
        rs.push_back(SiteReq{q.env, q.r, q.c, q.n, false});
      } else {
        PE_REQUIRE(q.env->col != nullptr, w + "dir 1 needs an environment built with PEPS_OPTS_COLUMNS");
        rs.push_back(SiteReq{q.env->col.get(), q.c, q.r, q.n, true});   // column c of the lattice
      }
    }
    dev::set_device(ctx->c->device);
    std::vector<peps_env*> es;
    std::vector<double> f0;
    for (const SiteReq& q : rs)
      if (std::find(es.begin(), es.end(), q.e) == es.end()) {
        es.push_back(q.e);
        f0.push_back(q.e->flops);
      }
    std::vector<double> lz, sg;
    double fl = 0.0;
    try {
      plan_site_env(*ctx->c, rs, lz, sg, fl);
    } catch (...) {
      for (size_t k = 0; k < es.size(); ++k) es[k]->flops = f0[k];
      throw;
    }
    for (size_t k = 0; k < es.size(); ++k) {   // the row sandwiches' flops are this call's, not the environment's
      fl += es[k]->flops - f0[k];
      es[k]->flops = f0[k];
    }
    for (int i = 0; i < n_req; ++i) {
      req[i].log_z = lz[i];
      req[i].sign = sg[i];
    }
    if (flops) *flops = fl;
  });
}

peps_status peps_env_info(peps_env* env, int32_t* n_rows, int32_t* max_halfsweeps, double* omegas, int32_t* sweeps,
                          int32_t* n_unconverged) {
  return guarded([&] {
    PE_REQUIRE(env != nullptr, "env must not be NULL");
    std::vector<const Mps*> rows;
    for (const std::vector<Mps>* v : {&env->top, &env->bot})
      for (size_t k = 1; k < v->size(); ++k)
        if ((*v)[k].truncated) rows.push_back(&(*v)[k]);
    int hmax = 0, unconv = 0;
    for (const Mps* m : rows) {
      hmax = std::max(hmax, m->n_omega);
      unconv += m->converged ? 0 : 1;
    }
    if (n_rows) *n_rows = (int32_t)rows.size();
    if (max_halfsweeps) *max_halfsweeps = hmax;
    if (n_unconverged) *n_unconverged = unconv;
    for (size_t i = 0; i < rows.size(); ++i) {
      if (sweeps) sweeps[i] = rows[i]->n_omega;
      if (omegas) {
        double* o = omegas + i * (size_t)hmax;
        for (int h = 0; h < hmax; ++h) o[h] = std::nan("");
        dev::set_device(env->ctx->device);
        dev::d2h(o, rows[i]->omega, sizeof(double) * rows[i]->n_omega, env->ctx->stream);
      }
    }
    if (omegas && !rows.empty()) dev::sync(env->ctx->stream);
  });
}

peps_status peps_env_mps(peps_env* env, int32_t side, int32_t k, int32_t c, int32_t* dims, double* dst,
                         double* log_scale) {
  return guarded([&] {
    PE_REQUIRE(env != nullptr, "env must not be NULL");
    PE_REQUIRE(side >= 0 && side <= 3, "side must be 0..3");
    peps_env* e = env;
    if (side >= 2) {
      PE_REQUIRE(env->col != nullptr, "sides 2 and 3 need an environment built with PEPS_OPTS_COLUMNS");
      e = env->col.get();
    }
    const std::vector<Mps>& v = (side & 1) == 0 ? e->top : e->bot;
    PE_REQUIRE(k >= 1 && k < (int)v.size(), "k must be in [1, rows)");
    const Mps& m = v[k];
    PE_REQUIRE(c >= 0 && c < (int)m.leg.size(), "c outside the boundary");
    const int32_t d[4] = {m.bond[c], m.leg[c], m.leg[c], m.bond[c + 1]};
    if (dims) std::memcpy(dims, d, sizeof(d));
    if (log_scale) *log_scale = ((side & 1) == 0 ? e->top_log : e->bot_log)[k];
    if (dst) {
      dev::set_device(env->ctx->device);
      dev::d2d(dst, m.t64[c], sizeof(double) * (size_t)d[0] * d[1] * d[2] * d[3], env->ctx->stream);
      dev::sync(env->ctx->stream);
    }
  });
}

peps_status peps_qr(peps_ctx* ctx, const peps_qr_block* blk, int32_t n_blocks) {
  return guarded([&] {
    PE_REQUIRE(ctx && blk, "ctx and blk must not be NULL");
    PE_REQUIRE(n_blocks >= 1, "n_blocks must be >= 1");
    for (int i = 0; i < n_blocks; ++i) {
      const peps_qr_block& b = blk[i];
      const std::string w = "block " + std::to_string(i) + ": ";
      PE_REQUIRE(b.a && b.q, w + "a and q must not be NULL");
      PE_REQUIRE(b.n >= 1 && b.m >= b.n && b.n <= 1024, w + "needs m >= n >= 1 and n <= 1024");
    }
    dev::set_device(ctx->c->device);
    Arena call(&ctx->c->pool);
    Rec rec(ctx->c.get(), &call);
    std::vector<QrDesc> ds;
    for (int i = 0; i < n_blocks; ++i) {
      const peps_qr_block& b = blk[i];
      double* w = (double*)call.alloc(sizeof(double) * 2 * (size_t)b.m * b.n);   // streaming-kernel workspace
      ds.push_back(QrDesc{b.a, b.a_rs, b.a_cs, b.q, b.q_rs, b.q_cs, b.r, b.r_rs, b.r_cs, w, b.m, b.n});
    }
    rec.qr(ds);
    rec.run(call);
  });
}

peps_status peps_ctx_autotune(peps_ctx* ctx, int32_t mode) {
  return guarded([&] {
    PE_REQUIRE(ctx != nullptr, "ctx must not be NULL");
    PE_REQUIRE(mode >= 0 && mode <= 2, "mode must be 0, 1 or 2");
    if (mode == 2) ctx->c->tuned.clear();
    ctx->c->tuning = mode == 1;
  });
}

peps_status peps_ctx_graphs(peps_ctx* ctx, int32_t enable) {
  return guarded([&] {
    PE_REQUIRE(ctx != nullptr, "ctx must not be NULL");
    dev::set_device(ctx->c->device);
    if (!enable && ctx->c->graphs) {
      dev::sync(ctx->c->stream);
      ctx->c->clear_graphs();
    }
    ctx->c->graphs = enable != 0;
  });
}

peps_status peps_ctx_profile(peps_ctx* ctx, int32_t enable) {
  return guarded([&] {
    PE_REQUIRE(ctx != nullptr, "ctx must not be NULL");
    ctx->c->profile = enable != 0;
    for (int i = 0; i < Ctx::NSTAT; ++i) {
      ctx->c->st_flops[i] = 0.0;
      ctx->c->st_bytes[i] = 0.0;
      ctx->c->st_ms[i] = 0.0;
      ctx->c->st_launch[i] = 0;
    }
  });
}

static_assert(Ctx::NSTAT == PEPS_N_STATS, "statistics table size is part of the ABI");

peps_status peps_ctx_stats(peps_ctx* ctx, double* flops, double* ms, int64_t* launches, double* bytes) {
  return guarded([&] {
    PE_REQUIRE(ctx && flops && ms && launches, "arguments must not be NULL");
    for (int i = 0; i < Ctx::NSTAT; ++i) {
      if (bytes) bytes[i] = ctx->c->st_bytes[i];
      flops[i] = ctx->c->st_flops[i];
      ms[i] = ctx->c->st_ms[i];
      launches[i] = ctx->c->st_launch[i];
    }
  });
}

peps_status peps_ctx_set_workspace(peps_ctx* ctx, uint64_t bytes) {
  return guarded([&] {
    PE_REQUIRE(ctx != nullptr, "ctx must not be NULL");
    PE_REQUIRE(bytes >= (uint64_t(1) << 20), "workspace budget below 1 MiB");
    ctx->c->scratch_budget = bytes;
  });
}

}  // extern "C"
