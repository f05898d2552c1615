// Host runtime of libpepsenv: memory pool, op recorder, tensor views and the
// environment data structures.
#pragma once
#include <initializer_list>
#include <map>
#include <memory>
#include <unordered_map>

#include "devapi.hpp"
#include "kernels.hpp"

namespace pe {

// ---------------------------------------------------------------- memory ----
// Caching device allocator: freed blocks are kept per size class and handed
// out again, so repeated calls with the same shapes allocate nothing.
class Pool {
 public:
  ~Pool();
  void* alloc(size_t bytes);
  void release(void* p);
  void trim();
  size_t bytes_in_use() const { return in_use_; }

 private:
  std::unordered_map<size_t, std::vector<void*>> free_;   // per size class
  std::unordered_map<void*, size_t> size_of_;
  size_t in_use_ = 0;
};

// Allocations of one object (environment or call), returned to the pool on
// destruction.
class Arena {
 public:
  explicit Arena(Pool* p) : pool_(p) {}
  // A fixed device region handed out by bumping an offset (256-byte
  // aligned); a request beyond its end throws OOM.  Nothing is allocated.
  Arena(void* base, size_t cap) : base_((uint8_t*)base), cap_(cap) {}
  ~Arena() { clear(); }
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  void* alloc(size_t bytes) {
    if (!pool_) {
      const size_t off = (used_ + 255) & ~size_t(255);
      if (off > cap_ || bytes > cap_ - off)
        throw Error(ST_OOM, "request needs more than the " + std::to_string(cap_) + "-byte fixed workspace");
      used_ = off + bytes;
      return base_ + off;
    }
    void* p = pool_->alloc(bytes);
    blocks_.push_back(p);
    return p;
  }
  void clear() {
    if (!pool_) {
      used_ = 0;
      return;
    }
    for (void* p : blocks_) pool_->release(p);
    blocks_.clear();
  }
  size_t used() const { return used_; }
  // Take over the blocks of `o` (an arena on the same pool), leaving it empty.
  void adopt(Arena& o) {
    PE_REQUIRE(pool_ && o.pool_ == pool_, "arenas of different pools");
    blocks_.insert(blocks_.end(), o.blocks_.begin(), o.blocks_.end());
    o.blocks_.clear();
  }

 private:
  Pool* pool_ = nullptr;
  std::vector<void*> blocks_;
  uint8_t* base_ = nullptr;
  size_t cap_ = 0, used_ = 0;
};

// A vector of at most N elements held in place: the dimensions and strides
// of views and the sub-dimension lists of descriptors, formed by the
// hundred thousand per batched call, cost no heap allocation.
template <class T, int N>
struct SmallVec {
  T v[N];
  int n = 0;
  SmallVec() = default;
  SmallVec(std::initializer_list<T> l) {
    for (const T& x : l) push_back(x);
  }
  SmallVec(const std::vector<T>& l) {
    for (const T& x : l) push_back(x);
  }
  size_t size() const { return (size_t)n; }
  bool empty() const { return n == 0; }
  T& operator[](size_t i) { return v[i]; }
  const T& operator[](size_t i) const { return v[i]; }
  T* begin() { return v; }
  T* end() { return v + n; }
  const T* begin() const { return v; }
  const T* end() const { return v + n; }
  T& back() { return v[n - 1]; }
  void push_back(const T& x) {
    PE_REQUIRE(n < N, "more than " + std::to_string(N) + " entries in a fixed-capacity list");
    v[n++] = x;
  }
  void assign(size_t k, const T& x) {
    n = 0;
    for (size_t i = 0; i < k; ++i) push_back(x);
  }
  void clear() { n = 0; }
  bool operator==(const SmallVec& o) const {
    if (n != o.n) return false;
    for (int i = 0; i < n; ++i)
      if (!(v[i] == o.v[i])) return false;
    return true;
  }
  bool operator!=(const SmallVec& o) const { return !(*this == o); }
};
using Dims = SmallVec<int64_t, 12>;

// ------------------------------------------------------------------ views ---
// A strided tensor view with one character label per index.
struct TV {
  const void* p = nullptr;
  int dt = DT_F64;
  std::string idx;
  Dims dim, str;
  int64_t size() const {
    int64_t n = 1;
    for (auto d : dim) n *= d;
    return n;
  }
};
TV dense(const void* p, int dt, const std::string& idx, const Dims& dims);
TV relabel(TV v, const std::string& idx);
// C = alpha * contraction(X, Y) + beta * C, every index in exactly two views.
TcDesc tc_build(const TV& C, const TV& X, const TV& Y, double alpha = 1.0, double beta = 0.0);
// Y = (X contracted with the ket site K) contracted with the bra site B in one
// fused launch (see KbDesc); kb_fits tells whether the kernel takes it.
KbDesc kb_build(const TV& Y, const TV& X, const TV& K, const TV& B);
bool kb_fits(const KbDesc& d, int prec);
double kb_flops(const KbDesc& d);

// --------------------------------------------------------------- recorder ---
// Records grouped launches and their descriptors, then uploads every
// descriptor in one copy and issues the launches in order on one stream.
struct Ctx;
class Rec {
 public:
  // `scratch` (optional) provides record-time workspace, e.g. split-K partials.
  explicit Rec(Ctx* c, Arena* scratch = nullptr);
  // Plain issue: no graph capture, profiling events, autotuning or pinned
  // staging (descriptors are copied from host memory and waited for), so
  // that with fixed arenas the recorder allocates no device or pinned memory.
  void set_plain() { plain_ = true; }
  // Whether a QR group whose largest block is mm x nn runs on the streaming
  // kernel, the only route that reads the blocks' workspace W.
  static bool qr_streaming(int mm, int nn) { return qr_variant_for(mm, nn) < 0 && nn > TSQR_NMAX; }
  void tc(int prec, int out_dt, std::vector<TcDesc> ds, bool algorithmic = true);
  void kb(int prec, int out_dt, std::vector<KbDesc> ds, bool algorithmic = true);
  // Fused two-row column steps (float64); `flops` their algorithmic flops.
  void k2(std::vector<K2Desc> ds, double flops);
  // Fused one-row chain steps (float64); `flops` their algorithmic flops.
  void kc(std::vector<KcDesc> ds, double flops);
  // Short, skinny FP64 contractions (see TskDesc).
  void tsk(std::vector<TskDesc> ds, bool algorithmic);
  void qr(const std::vector<QrDesc>& ds);
  void reduce(std::vector<RedDesc> ds);
  void ew(std::vector<EwDesc> ds);
  void sep(const std::vector<SepDesc>& ds);
  // Device copy of host data, available to every op recorded after this call.
  void* aux(Arena& arena, const void* data, size_t bytes);
  // Upload and launch everything recorded so far (no wait).  Device memory
  // for descriptors comes from `arena`, which must outlive the stream work.
  void flush(Arena& arena);
  // flush(), wait for the stream, collect profiling statistics.
  void run(Arena& arena);
  ~Rec();
  double flops() const { return flops_; }

 private:
  struct Op {
    int kind, prec, out_dt, tile, nd, grid;
    size_t off;
    double flops;
    int ksm = 0, kp = 0;   // skinny contraction: k-steps per load batch, padded K (fused: padded lu, p*q)
    int q = 0;             // fused contraction: largest q
    double bytes = 0.0;    // algorithmic bytes: operands read once, output written once
  };
  size_t push_bytes(const void* p, size_t n);
  void issue(const uint8_t* dblob, double* partials, unsigned* counters, bool timed, hipStream_t s);
  void flush_graph();
  void tc_launch(int prec, int out_dt, int tile, std::vector<TcDesc> ds, bool algorithmic, bool allow_split);
  void apply_choice(int prec, int out_dt, int fam, int choice, std::vector<TcDesc> ds, bool algorithmic);
  int tune(int prec, int out_dt, int fam, bool skinny, const std::vector<TcDesc>& ds, uint64_t key);
  bool tcs_launch(int prec, int out_dt, std::vector<TcDesc>& ds, bool algorithmic);
  void qr_tall(const std::vector<QrDesc>& ds);
  void qr_cq(const std::vector<QrDesc>& ds, int nb);
  double* qr_scratch(size_t n);
  static constexpr int TSQR_LEAF = 256, TSQR_NMAX = 80;   // leaf rows, widest tree-factored block
  double* qr_buf_ = nullptr;   // TSQR workspace (scratch), reused by every QR op of this recorder
  size_t qr_cap_ = 0, qr_used_ = 0;
  int qr_depth_ = 0;
  Ctx* ctx_;
  Arena* scratch_;
  bool plain_ = false;
  std::vector<Op> ops_;
  std::vector<uint8_t> blob_;
  std::vector<std::pair<void*, std::pair<size_t, size_t>>> aux_;   // dst, (blob offset, bytes)
  int partials_ = 0;
  int cq_slots_ = 0;             // arrival counters of this recording (CholeskyQR2, skinny split-K; zeroed at issue)
  double* part_buf_ = nullptr;   // split-K partial tiles (scratch)
  size_t part_cap_ = 0;
  double flops_ = 0.0;
  std::vector<std::pair<void*, size_t>> pinned_;   // staging buffers in flight
  struct Timed {
    void *e0, *e1;
    int key;
    double flops, bytes;
  };
  std::vector<Timed> events_;
};

// ---------------------------------------------------------------- context ---
struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  Pool pool;
  size_t scratch_budget = size_t(48) << 30;
  bool profile = false;
  static constexpr int NSTAT = 3 * 2 * TT_COUNT;
  double st_flops[NSTAT] = {0};
  double st_bytes[NSTAT] = {0};
  double st_ms[NSTAT] = {0};
  int64_t st_launch[NSTAT] = {0};
  // launch shapes chosen by timing (see Rec::tune), by group signature
  bool tuning = false;
  std::unordered_map<uint64_t, int> tuned;
  // replayable launch sequences (see Rec::flush_graph)
  bool graphs = false;
  struct Graph {
    std::vector<uint8_t> key;
    void* exec = nullptr;
    uint8_t* dblob = nullptr;
    double* partials = nullptr;
    unsigned* counters = nullptr;
  };
  static constexpr int GRAPH_MAX = 512;
  std::unordered_map<uint64_t, std::vector<Graph>> graph_cache;
  int graph_count = 0;
  hipStream_t capture_stream = nullptr;   // graphs are recorded here (the caller's may be the null stream)
  void clear_graphs();
  std::vector<uint8_t> blob_spare;              // a recorder's descriptor buffer, kept for the next one
  std::multimap<size_t, void*> pinned_free;     // pinned staging buffers by capacity
  std::unordered_map<void*, size_t> pinned_size;
  ~Ctx();
  void* pinned_get(size_t bytes);
  void pinned_put(void* p, size_t bytes);
};

// ----------------------------------------------------------- environment ---
// Packed site tensor: copies in the contraction dtype with the identity,
// S^z, S^+ and S^- applied to the ket physical leg.
struct Site {
  void* op[4] = {nullptr, nullptr, nullptr, nullptr};
  int d = 2, Dl = 1, Du = 1, Dr = 1, Dd = 1;
  // A site of the transposed lattice (left/right legs exchanged with up/down
  // ones) that shares the buffers of the original site: they hold the legs
  // in the order (p, u, l, d, r) of this view.
  bool tr = false;
};

struct Lattice {
  int Lr = 0, Lc = 0;
  std::vector<const Site*> s;                 // row-major
  std::vector<const void*> lam, rho, tau, beta;   // closings in the compute dtype
  const Site& at(int r, int c) const { return *s[(size_t)r * Lc + c]; }
};

// Boundary MPS: Lc tensors [a][k][b][a'] in float64 and in the compute dtype.
struct Mps {
  std::vector<double*> t64;
  std::vector<const void*> tc;
  std::vector<int> bond;   // Lc+1 entries, bond[0] = bond[Lc] = 1
  std::vector<int> leg;    // Lc entries
  const double* omega = nullptr;   // device slots of the squared centre norms (null: closing)
  int n_omega = 0;                 // 1 for an exact row, the half-sweeps run for a truncated one
  bool truncated = false;
  bool converged = true;           // false: stopped at max_halfsweeps before the tolerance
};

struct Opts {
  int chi = 1, dtype = 0, halfsweeps = 4;
  int max_halfsweeps = 4;   // > halfsweeps only with tol > 0
  double tol = 0.0;         // relative change of the squared centre norm that ends the ALS sweeps
  bool strict = false;      // an unconverged row fails the call
  uint64_t seed = 0;
  bool columns = false;   // also the left and right boundaries
  int prec() const { return dtype; }
  int cdt() const { return dtype == 0 ? DT_F64 : DT_F32; }
};

}  // namespace pe

// The context's state is shared with every environment made from it, so an
// environment stays valid (and frees into a live pool) even if the context
// handle is destroyed first.
struct peps_ctx {
  std::shared_ptr<pe::Ctx> c;
};

struct peps_env {
  explicit peps_env(const std::shared_ptr<pe::Ctx>& c) : ctxref(c), ctx(c.get()), arena(&c->pool) {}
  std::shared_ptr<pe::Ctx> ctxref;   // declared first: released last
  pe::Ctx* ctx;
  pe::Arena arena;
  pe::Opts opts;
  pe::Lattice lat;
  std::vector<std::unique_ptr<pe::Site>> sites;   // owned packed sites (may be shared by windows)
  std::shared_ptr<void> shared_owner;             // keeps a parent's packed data alive
  std::vector<pe::Mps> top;   // top[k] = T_{k-1}: rows 0..k-1 absorbed, k = 0..Lr-1
  std::vector<pe::Mps> bot;   // bot[k]: rows Lr-k..Lr-1 absorbed (flipped frame)
  std::vector<double> top_log, bot_log;   // cumulative log-scales (accumulated on the device, FP64)
  bool window = false;
  int ci = 0, cj = 0;                     // centre (window coordinates)
  double flops = 0.0;
  // Left and right boundaries, as the top and bottom boundaries of the
  // transposed lattice (its sites are views of this lattice's buffers);
  // peps_expect then takes the vertical bonds from its single-row sandwiches.
  std::unique_ptr<peps_env> col;
  int side0 = 0;   // ALS start-stream side of the top boundaries (bottom: side0 + 1)
  // Single-row sandwiches (column environments in this environment's
  // memory) of rows already used by site, bond or fit calls, by row.
  std::map<int, std::shared_ptr<void>> row_env;
  pe::Mps& T(int r) { return top[r + 1]; }
  pe::Mps& B(int r) { return bot[lat.Lr - r]; }
  double Tlog(int r) const { return top_log[r + 1]; }
  double Blog(int r) const { return bot_log[lat.Lr - r]; }
};
