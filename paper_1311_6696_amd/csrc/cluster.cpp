// Cluster environments (arXiv:1311.6696, Sec. 5): outside an n x n window
// around a site the environment is the positive separable (D' = 1) boundary
// of CU_0 (Sec. 5.1, figs. SepEnv1/SepEnv2), inside it the sandwich
// contraction with bond chi runs as for a whole lattice (Sec. 5.2, 5.3).
//
// The separable boundaries of the four directions are computed once per
// lattice (one workgroup per direction); every window then becomes an
// environment whose cut legs are closed by them, and all windows run through
// the batched boundary planner together.
#include <array>
#include <functional>

#include "../../include/peps_env.h"
#include "chains.hpp"

namespace pe {
namespace {

struct ClusterData {
  explicit ClusterData(Ctx* c) : arena(&c->pool) {}
  Arena arena;
  std::vector<std::vector<std::unique_ptr<Site>>> sites;   // per state
  void* one = nullptr;
  struct Dir {
    int Lr = 0, Lc = 0;
    double* sig64 = nullptr;
    void* sigc = nullptr;
    std::vector<int64_t> off;
    int32_t* sweeps = nullptr;
    double* delta = nullptr;
  };
  std::vector<std::array<Dir, 4>> dirs;   // per state: top, bottom, left, right frames
};

// Frame (k, c) of direction `dir` -> original site and leg permutation.
// top: as given; bottom: rows mirrored, u <-> d; left: rows <-> columns
// (l <-> u, r <-> d); right: the left frame mirrored.
void frame_map(const peps_state& st, int dir, int k, int c, int& r, int& cc, int map[5]) {
  static const int MAPS[4][5] = {{0, 1, 2, 3, 4}, {0, 1, 4, 3, 2}, {0, 2, 1, 4, 3}, {0, 2, 3, 4, 1}};
  for (int i = 0; i < 5; ++i) map[i] = MAPS[dir][i];
  switch (dir) {
    case 0: r = k; cc = c; break;
    case 1: r = st.rows - 1 - k; cc = c; break;
    case 2: r = c; cc = k; break;
    default: r = c; cc = st.cols - 1 - k; break;
  }
}

SepSite frame_site(const peps_state& st, int dir, int k, int c) {
  int r, cc, map[5];
  frame_map(st, dir, k, c, r, cc, map);
  const int32_t* o = st.dims + 5 * ((size_t)r * st.cols + cc);
  int64_t s[5];
  s[4] = 1;
  for (int i = 3; i >= 0; --i) s[i] = s[i + 1] * o[i + 1];
  SepSite f;
  f.A = st.site[(size_t)r * st.cols + cc];
  int32_t* fd[5] = {&f.d, &f.Dl, &f.Du, &f.Dr, &f.Dd};
  int64_t* fs[5] = {&f.sp, &f.sl, &f.su, &f.sr, &f.sd};
  for (int i = 0; i < 5; ++i) {
    *fd[i] = o[map[i]];
    *fs[i] = s[map[i]];
  }
  f.pad = 0;
  return f;
}

}  // namespace
}  // namespace pe

using namespace pe;

// Defined in capi.cpp.
namespace pe {
void validate_state_public(const peps_state& s, int idx);
void check_finite_public(Ctx& C, const peps_state* st, int n_states, const std::vector<char>& used);
Opts make_opts_public(const peps_env_opts* o);
std::unique_ptr<peps_env> transposed_env_public(const peps_env& e);
void pack_state_public(Rec& rec, Arena& arena, const peps_state& s, int cdt, std::vector<std::unique_ptr<Site>>& out);
void* make_one_public(Rec& rec, Arena& arena, int cdt);
peps_status guarded_public(const std::function<void()>& f);
}  // namespace pe

extern "C" peps_status peps_cluster_env(peps_ctx* ctx, const peps_state* st, int32_t n_states, const peps_window* win,
                                        int32_t n_win, const peps_env_opts* opts, peps_env** out) {
  std::vector<peps_env*> made;
  peps_status status = guarded_public([&] {
    PE_REQUIRE(ctx && st && win && out, "ctx, st, win and out must not be NULL");
    PE_REQUIRE(n_states >= 1 && n_win >= 1, "n_states and n_win must be >= 1");
    const Opts o = make_opts_public(opts);
    for (int i = 0; i < n_states; ++i) validate_state_public(st[i], i);
    std::vector<char> used(n_states, 0);
    for (int w = 0; w < n_win; ++w) {
      const peps_window& x = win[w];
      const std::string at = "window " + std::to_string(w) + ": ";
      PE_REQUIRE(x.state >= 0 && x.state < n_states, at + "state index out of range");
      const peps_state& s = st[x.state];
      PE_REQUIRE(0 <= x.r0 && x.r0 <= x.ci && x.ci <= x.r1 && x.r1 < s.rows, at + "rows out of range");
      PE_REQUIRE(0 <= x.c0 && x.c0 <= x.cj && x.cj <= x.c1 && x.c1 < s.cols, at + "columns out of range");
      used[x.state] = 1;
    }
    for (int i = 0; i < n_states; ++i) {
      if (!used[i]) continue;
      for (int k = 0; k < 5 * st[i].rows * st[i].cols; ++k)
        if (k % 5 != 0 && st[i].dims[k] > SEP_MAXD)
          throw Error(ST_UNSUPPORTED, "cluster environments support virtual bonds up to " + std::to_string(SEP_MAXD));
    }
    dev::set_device(ctx->c->device);
    Ctx& C = *ctx->c;
    check_finite_public(C, st, n_states, used);
    auto data = std::make_shared<ClusterData>(&C);
    Arena tmp(&C.pool);
    Rec rec(&C);
    const int cdt = o.cdt();
    data->sites.resize(n_states);
    data->dirs.resize(n_states);
    data->one = make_one_public(rec, data->arena, cdt);
    std::vector<SepDesc> seps;
    std::vector<EwDesc> casts;
    for (int i = 0; i < n_states; ++i) {
      if (!used[i]) continue;
      pack_state_public(rec, data->arena, st[i], cdt, data->sites[i]);
      for (int dir = 0; dir < 4; ++dir) {
        ClusterData::Dir& D = data->dirs[i][dir];
        D.Lr = dir < 2 ? st[i].rows : st[i].cols;
        D.Lc = dir < 2 ? st[i].cols : st[i].rows;
        if (D.Lr < 2) continue;
        std::vector<SepSite> fs;
        int64_t tot = 0;
        int dmax = 1;
        for (int k = 0; k < D.Lr; ++k)
          for (int c = 0; c < D.Lc; ++c) {
            fs.push_back(frame_site(st[i], dir, k, c));
            const SepSite& q = fs.back();
            PE_REQUIRE(q.d <= 2, "CU_0 boundaries need physical dimension <= 2");
            dmax = std::max({dmax, q.Dl, q.Du, q.Dr, q.Dd});
            if (k + 1 < D.Lr) {
              D.off.push_back(tot);
              tot += (int64_t)fs.back().Dd * fs.back().Dd;
            }
          }
        D.sig64 = (double*)data->arena.alloc(sizeof(double) * tot);
        D.sigc = cdt == DT_F64 ? (void*)D.sig64 : data->arena.alloc(4 * tot);
        D.sweeps = (int32_t*)tmp.alloc(sizeof(int32_t) * D.Lr);
        D.delta = (double*)tmp.alloc(sizeof(double) * D.Lr);
        SepDesc sd;
        std::memset(&sd, 0, sizeof(sd));
        sd.Lr = D.Lr;
        sd.Lc = D.Lc;
        sd.max_sweeps = 500;
        sd.dmax = dmax;
        sd.tol = 1e-14;
        sd.sites = (const SepSite*)rec.aux(tmp, fs.data(), fs.size() * sizeof(SepSite));
        sd.off = (const int64_t*)rec.aux(tmp, D.off.data(), D.off.size() * sizeof(int64_t));
        sd.sig = D.sig64;
        const size_t V = SEP_MAXD * SEP_MAXD;
        sd.work = (double*)tmp.alloc(sizeof(double) * ((3 * (size_t)D.Lc + 3) * V + 2 * V * V));
        sd.sweeps = D.sweeps;
        sd.delta = D.delta;
        seps.push_back(sd);
        if (cdt != DT_F64) casts.push_back(ew_desc(EW_COPY, D.sig64, DT_F64, D.sigc, DT_F32, tot));
      }
    }
    rec.sep(seps);
    rec.ew(std::move(casts));
    rec.run(tmp);
    // window environments
    auto sigma = [&](int i, int dir, int k, int c) -> const void* {
      const ClusterData::Dir& D = data->dirs[i][dir];
      const char* base = (const char*)D.sigc;
      return base + dtype_size(cdt) * D.off[(size_t)k * D.Lc + c];
    };
    for (int w = 0; w < n_win; ++w) {
      const peps_window& x = win[w];
      const int i = x.state;
      const peps_state& s = st[i];
      auto* e = new peps_env(ctx->c);
      made.push_back(e);
      e->opts = o;
      e->window = true;
      e->ci = x.ci - x.r0;
      e->cj = x.cj - x.c0;
      e->shared_owner = data;
      Lattice& L = e->lat;
      L.Lr = x.r1 - x.r0 + 1;
      L.Lc = x.c1 - x.c0 + 1;
      for (int r = x.r0; r <= x.r1; ++r)
        for (int c = x.c0; c <= x.c1; ++c) L.s.push_back(data->sites[i][(size_t)r * s.cols + c].get());
      for (int r = x.r0; r <= x.r1; ++r) {
        L.lam.push_back(x.c0 == 0 ? data->one : sigma(i, 2, x.c0 - 1, r));
        L.rho.push_back(x.c1 == s.cols - 1 ? data->one : sigma(i, 3, s.cols - 2 - x.c1, r));
      }
      for (int c = x.c0; c <= x.c1; ++c) {
        L.tau.push_back(x.r0 == 0 ? data->one : sigma(i, 0, x.r0 - 1, c));
        L.beta.push_back(x.r1 == s.rows - 1 ? data->one : sigma(i, 1, s.rows - 2 - x.r1, c));
      }
      if (o.columns) {   // the transposed window: its centre row is the centre's column
        e->col = transposed_env_public(*e);
        e->col->window = true;
        e->col->ci = e->cj;
        e->col->cj = e->ci;
      }
    }
    std::vector<peps_env*> all(made);
    for (peps_env* e : made)
      if (e->col) all.push_back(e->col.get());
    plan_boundaries(C, all);
    for (int w = 0; w < n_win; ++w) out[w] = made[w];
  });
  if (status != PEPS_OK) {
    for (peps_env* e : made) delete e;
    if (out && n_win > 0)
      for (int w = 0; w < n_win; ++w) out[w] = nullptr;
  }
  return status;
}
