// Planning of the boundary contraction, the sandwiches and the clusters.
#pragma once
#include "runtime.hpp"

namespace pe {

// Record-time scratch allocator: a block returned with put() may be handed
// out again to ops recorded later (all ops run in record order on one
// stream).  Memory comes from an arena that outlives the run.
class Scratch {
 public:
  explicit Scratch(Arena& a) : arena_(a) {}
  void* get(size_t bytes);
  void put(void* p);
  size_t held() const { return held_; }

 private:
  Arena& arena_;
  std::map<size_t, std::vector<void*>> free_;   // by exact size
  std::unordered_map<void*, size_t> size_;
  size_t held_ = 0;
};

// Top and bottom boundaries of every environment (one batched run).
void plan_boundaries(Ctx& ctx, std::vector<peps_env*>& envs);

// Observables of every environment (one batched run); results on the host.
struct ExpectOut {
  double log_norm = 0.0, sign = 1.0;
  std::vector<double> sz, bond;
};
void plan_expect(Ctx& ctx, std::vector<peps_env*>& envs, std::vector<ExpectOut>& out);

// Norm environments of single sites (one batched run): site (r, c) of e
// (window coordinates for a window), written as a float64 matrix into the
// device buffer `out`, scaled so that sum_p A N A = sign; log|<psi|psi>| as
// that row's sandwich estimates it, the sign, and the algorithmic flops of
// the environment chains on the host.
struct SiteReq {
  peps_env* e;
  int r, c;
  double* out;
  bool tr = false;   // e is a transposed lattice: write N in the original site's leg order
};
void plan_site_env(Ctx& ctx, std::vector<SiteReq>& req, std::vector<double>& log_z, std::vector<double>& sign,
                   double& flops);

// Right-hand sides b of the ALS update of the horizontal bond (r,c)-(r,c+1)
// under a two-site gate (one batched run): b of either site (device float64
// [p][l][u][r][d], may be null) in the scaling of that site's norm
// environment; algorithmic flops on the host.
struct BondReq {
  peps_env* e;
  int r, c;
  const double* gate;   // device, d^2 x d^2 float64
  double* bl;
  double* br;
  bool tr = false;   // e is a transposed lattice (a vertical bond): b in the original leg order
};
void plan_bond_env(Ctx& ctx, std::vector<BondReq>& req, double& flops);

// The bond update's two local problems with substitute site tensors (one
// batched run, float64 environments): N1, b1 of the first site with the
// second replaced by s2, N2, b2 of the second with the first replaced by s1,
// in the gated bond's scaling (device float64 outputs, sites' own order).
struct FitReq {
  peps_env* e;
  int r, c;
  const double* gate;
  const double* s1;
  const double* s2;
  double* n1;
  double* b1;
  double* n2;
  double* b2;
  bool tr = false;
};
void plan_bond_fit(Ctx& ctx, std::vector<FitReq>& req, double& flops);

// <X|Y>, <X|X>, <Y|Y> of pairs of stored boundaries of one row (float64
// tensors, (ket, bra) taken as one physical index), one batched run.
struct OvReq {
  const Mps* x;
  const Mps* y;
  double out[3];
};
void plan_overlap(Ctx& ctx, std::vector<OvReq>& req);

}  // namespace pe
