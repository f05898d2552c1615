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
  std::multimap<size_t, void*> free_;
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

}  // namespace pe
