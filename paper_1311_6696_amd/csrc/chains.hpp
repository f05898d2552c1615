// Stage builders shared by the boundary, sandwich and cluster planners: each
// appends the descriptors of one job to per-stage vectors (one grouped
// launch per stage for a whole batch of jobs).
#pragma once
#include <algorithm>
#include <cmath>

#include "planner.hpp"

namespace pe {

constexpr int OP_ID = 0, OP_SZ = 1, OP_SP = 2, OP_SM = 3;
// Heisenberg bond S.S = Sz Sz + (S+ S- + S- S+)/2: (weight, first, second)
constexpr double BOND_W[3] = {1.0, 0.5, 0.5};
constexpr int BOND_O1[3] = {OP_SZ, OP_SP, OP_SM};
constexpr int BOND_O2[3] = {OP_SZ, OP_SM, OP_SP};

inline int64_t prod(const std::vector<int64_t>& v) {
  int64_t n = 1;
  for (auto x : v) n *= x;
  return n;
}

// Site view with labels "plurd"-like; flip swaps the up and down legs.  A
// transposed site is a strided view of the stored (p, u, l, d, r) order.
inline TV site_tv(const Site& s, int op, bool flip, int dt, const std::string& lbl) {
  TV v = s.tr ? dense(s.op[op], dt, lbl, {s.d, s.Du, s.Dl, s.Dd, s.Dr})
              : dense(s.op[op], dt, lbl, {s.d, s.Dl, s.Du, s.Dr, s.Dd});
  if (s.tr) {
    std::swap(v.dim[1], v.dim[2]);
    std::swap(v.str[1], v.str[2]);
    std::swap(v.dim[3], v.dim[4]);
    std::swap(v.str[3], v.str[4]);
  }
  if (flip) {
    std::swap(v.dim[2], v.dim[4]);
    std::swap(v.str[2], v.str[4]);
  }
  return v;
}

inline double tc_flops(const TcDesc& d) { return 2.0 * d.M * (double)d.N * d.K; }

// Per-stage descriptor lists of one batched chain (plain and fused ket-bra
// contractions); `flops` sums the algorithmic flops of every descriptor
// pushed.  `prec` decides whether a ket-bra pair may run fused.
struct St {
  std::vector<std::vector<TcDesc>> s;
  std::vector<std::vector<KbDesc>> k;
  std::vector<std::vector<KcDesc>> c;
  std::vector<double> cflops;
  double flops = 0.0;
  int prec = TP_F64;
  St(int n, int prec_) : s(n), k(n), c(n), cflops(n, 0.0), prec(prec_) {}
  void add(int stage, const TcDesc& d) {
    s[stage].push_back(d);
    flops += tc_flops(d);
  }
  void add_kb(int stage, const KbDesc& d) {
    k[stage].push_back(d);
    flops += kb_flops(d);
  }
  // Ket and bra of one site into `out` in one fused launch when the fused
  // kernel takes it (returns true); else nothing is added.
  bool add_fused(int stage, const TV& out, const TV& x, const TV& ket, const TV& bra) {
    const KbDesc d = kb_build(out, x, ket, bra);
    if (!kb_fits(d, prec)) return false;
    add_kb(stage, d);
    return true;
  }
  // The one-row chain of a site in one launch when the fused kernel takes it
  // (float64, D = 4, d = 2, a <= K2_CHI; returns true); `right`: the
  // right-to-left chain, whose horizontal legs swap roles.
  bool add_chain(int stage, const TV& out, const TV& E, const TV& T, const TV& Ak, const TV& Ab, int dt, bool right) {
    if (prec != TP_F64 || dt != DT_F64) return false;
    const Dims site{2, 4, 4, 4, 4};
    if (Ak.dim != site || Ab.dim != site || E.dim[1] != 4 || E.dim[2] != 4 || T.dim[1] != 4 || T.dim[2] != 4) return false;
    const int64_t A = E.dim[3], Ne = right ? T.dim[0] : T.dim[3];
    if (A > K2_CHI || A != (right ? T.dim[3] : T.dim[0])) return false;
    KcDesc d;
    std::memset(&d, 0, sizeof(d));
    d.E = (const double*)E.p;
    d.T = (const double*)T.p;
    d.s[0] = (const double*)Ak.p;
    d.s[1] = (const double*)Ab.p;
    d.Y = (double*)const_cast<void*>(out.p);
    const int h[4] = {3, 1, 2, 0}, hs[5] = {0, 3, 2, 1, 4};
    for (int i = 0; i < 4; ++i) {
      d.sE[i] = E.str[i];
      d.sT[i] = right ? T.str[h[i]] : T.str[i];
    }
    for (int i = 0; i < 5; ++i) {
      d.ss[0][i] = right ? Ak.str[hs[i]] : Ak.str[i];
      d.ss[1][i] = right ? Ab.str[hs[i]] : Ab.str[i];
    }
    for (int i = 0; i < 6; ++i) d.sY[i] = out.str[i];
    d.X = (int32_t)E.dim[0];
    d.A = (int32_t)A;
    d.Ne = (int32_t)Ne;
    c[stage].push_back(d);
    // algorithmic flops: the boundary product and the ket and bra layers
    const double f = (double)d.X * d.Ne * (2.0 * 256 * A + 32768.0);
    cflops[stage] += f;
    flops += f;
    return true;
  }
  void record(Rec& rec, int prec_, int cdt) {
    for (size_t i = 0; i < s.size(); ++i) {
      rec.kc(std::move(c[i]), cflops[i]);
      rec.tc(prec_, cdt, std::move(s[i]));
      rec.kb(prec_, cdt, std::move(k[i]));
    }
  }
};

// Y3[x][d][g][r][s][e] = sum E[x][l][m][a] T[a][u][v][e] Ak[p][l][u][r][d] Ab[p][m][v][s][g]
inline TV chain_left(St& st, const TV& E, const TV& T, const TV& Ak, const TV& Ab, void* P, void* Q, int dt) {
  const int64_t X = E.dim[0], Dl = E.dim[1], Du = T.dim[1], Ee = T.dim[3];
  const int64_t p = Ak.dim[0], Dr = Ak.dim[3], Dd = Ak.dim[4];
  TV f = dense(Q, dt, "xdgrse", {X, Dd, Dd, Dr, Dr, Ee});   // fused: ket and bra in one launch, into Q
  if (st.add_chain(0, f, E, T, Ak, Ab, dt, false)) return f;   // the whole chain in one launch
  TV y1 = dense(P, dt, "xlmuve", {X, Dl, Dl, Du, Du, Ee});
  st.add(0, tc_build(y1, E, T));
  if (st.add_fused(1, f, y1, Ak, Ab)) return f;
  TV z = dense(Q, dt, "xdrpmve", {X, Dd, Dr, p, Dl, Du, Ee});
  st.add(1, tc_build(z, y1, Ak));
  TV y3 = dense(P, dt, "xdgrse", {X, Dd, Dd, Dr, Dr, Ee});
  st.add(2, tc_build(y3, z, Ab));
  return y3;
}

// Y3[y][d][g][l][m][a] = sum F[y][r][s][e] T[a][u][v][e] Ak[p][l][u][r][d] Ab[p][m][v][s][g]
inline TV chain_right(St& st, const TV& F, const TV& T, const TV& Ak, const TV& Ab, void* P, void* Q, int dt) {
  const int64_t Y = F.dim[0], Dr = F.dim[1], Du = T.dim[1], Aa = T.dim[0];
  const int64_t p = Ak.dim[0], Dl = Ak.dim[1], Dd = Ak.dim[4];
  TV f = dense(Q, dt, "ydglma", {Y, Dd, Dd, Dl, Dl, Aa});
  if (st.add_chain(0, f, F, T, Ak, Ab, dt, true)) return f;   // the whole chain in one launch
  TV y1 = dense(P, dt, "yrsuva", {Y, Dr, Dr, Du, Du, Aa});
  st.add(0, tc_build(y1, F, T));
  if (st.add_fused(1, f, y1, Ak, Ab)) return f;
  TV z = dense(Q, dt, "ydlpsva", {Y, Dd, Dl, p, Dr, Du, Aa});
  st.add(1, tc_build(z, y1, Ak));
  TV y3 = dense(P, dt, "ydglma", {Y, Dd, Dd, Dl, Dl, Aa});
  st.add(2, tc_build(y3, z, Ab));
  return y3;
}

inline int64_t chain_scratch_P(int64_t X, int64_t Dl, int64_t Du, int64_t Ee, int64_t Dr, int64_t Dd) {
  return std::max(X * Dl * Dl * Du * Du * Ee, X * Dd * Dd * Dr * Dr * Ee);
}

// Two-row column transfer (rows 1 and 2 between T and B), left to right.
inline TV chain2_left(St& st, const TV& L, const TV& T, const TV& A1k, const TV& A1b, const TV& A2k, const TV& A2b,
               void* P, void* Q, int dt) {
  const int64_t X = L.dim[0], D2l = L.dim[1], D1l = L.dim[3];
  const int64_t Du = T.dim[1], Ee = T.dim[3];
  const int64_t p1 = A1k.dim[0], Dr1 = A1k.dim[3], Dd1 = A1k.dim[4];
  const int64_t p2 = A2k.dim[0], Dr2 = A2k.dim[3], Dd2 = A2k.dim[4];
  TV y1 = dense(P, dt, "xLMlmuve", {X, D2l, D2l, D1l, D1l, Du, Du, Ee});
  st.add(0, tc_build(y1, L, T));
  // both rows fused (ket and bra of a row in one launch, Q then P), or both
  // through the plain chain (P -> Q -> P -> Q -> P)
  TV y2q = dense(Q, dt, "xLMdgrse", {X, D2l, D2l, Dd1, Dd1, Dr1, Dr1, Ee});
  TV y3p = dense(P, dt, "xDGRSrse", {X, Dd2, Dd2, Dr2, Dr2, Dr1, Dr1, Ee});
  const KbDesc k1 = kb_build(y2q, y1, A1k, A1b), k2 = kb_build(y3p, y2q, A2k, A2b);
  if (kb_fits(k1, st.prec) && kb_fits(k2, st.prec)) {
    st.add_kb(1, k1);
    st.add_kb(3, k2);
    return y3p;
  }
  TV z1 = dense(Q, dt, "xLMdrpmve", {X, D2l, D2l, Dd1, Dr1, p1, D1l, Du, Ee});
  st.add(1, tc_build(z1, y1, A1k));
  TV y2 = dense(P, dt, "xLMdgrse", {X, D2l, D2l, Dd1, Dd1, Dr1, Dr1, Ee});
  st.add(2, tc_build(y2, z1, A1b));
  TV z2 = dense(Q, dt, "xDRqMgrse", {X, Dd2, Dr2, p2, D2l, Dd1, Dr1, Dr1, Ee});
  st.add(3, tc_build(z2, y2, A2k));
  TV y3 = dense(P, dt, "xDGRSrse", {X, Dd2, Dd2, Dr2, Dr2, Dr1, Dr1, Ee});
  st.add(4, tc_build(y3, z2, A2b));
  return y3;
}

inline TV chain2_right(St& st, const TV& R, const TV& T, const TV& A1k, const TV& A1b, const TV& A2k, const TV& A2b,
                void* P, void* Q, int dt) {
  const int64_t Y = R.dim[0], Dr2 = R.dim[1], Dr1 = R.dim[3];
  const int64_t Du = T.dim[1], Aa = T.dim[0];
  const int64_t p1 = A1k.dim[0], Dl1 = A1k.dim[1], Dd1 = A1k.dim[4];
  const int64_t p2 = A2k.dim[0], Dl2 = A2k.dim[1], Dd2 = A2k.dim[4];
  TV y1 = dense(P, dt, "yRSrsuva", {Y, Dr2, Dr2, Dr1, Dr1, Du, Du, Aa});
  st.add(0, tc_build(y1, R, T));
  TV y2q = dense(Q, dt, "yRSdglma", {Y, Dr2, Dr2, Dd1, Dd1, Dl1, Dl1, Aa});
  TV y3p = dense(P, dt, "yDGLMlma", {Y, Dd2, Dd2, Dl2, Dl2, Dl1, Dl1, Aa});
  const KbDesc k1 = kb_build(y2q, y1, A1k, A1b), k2 = kb_build(y3p, y2q, A2k, A2b);
  if (kb_fits(k1, st.prec) && kb_fits(k2, st.prec)) {
    st.add_kb(1, k1);
    st.add_kb(3, k2);
    return y3p;
  }
  TV z1 = dense(Q, dt, "yRSdlpsva", {Y, Dr2, Dr2, Dd1, Dl1, p1, Dr1, Du, Aa});
  st.add(1, tc_build(z1, y1, A1k));
  TV y2 = dense(P, dt, "yRSdglma", {Y, Dr2, Dr2, Dd1, Dd1, Dl1, Dl1, Aa});
  st.add(2, tc_build(y2, z1, A1b));
  TV z2 = dense(Q, dt, "yDLqSglma", {Y, Dd2, Dl2, p2, Dr2, Dd1, Dl1, Dl1, Aa});
  st.add(3, tc_build(z2, y2, A2k));
  TV y3 = dense(P, dt, "yDGLMlma", {Y, Dd2, Dd2, Dl2, Dl2, Dl1, Dl1, Aa});
  st.add(4, tc_build(y3, z2, A2b));
  return y3;
}

inline EwDesc ew_desc(int kind, const void* src, int sdt, void* dst, int ddt, int64_t n) {
  EwDesc e;
  std::memset(&e, 0, sizeof(e));
  e.kind = kind;
  e.src = src;
  e.src_dt = sdt;
  e.dst = dst;
  e.dst_dt = ddt;
  e.n = n;
  return e;
}

// Small FP64 result arrays spread over device buffers, gathered into one
// buffer by a single copy launch recorded ahead of the flush, so that the
// host reads all of them back with one transfer instead of one per array.
struct Gather {
  struct Item {
    const double* src;
    size_t off, n;
  };
  std::vector<Item> items;
  size_t total = 0;
  double* buf = nullptr;
  std::vector<double> host;
  size_t add(const double* d, size_t n) {
    items.push_back({d, total, n});
    total += n;
    return total - n;
  }
  void record(Rec& rec, Arena& arena) {
    if (!total) return;
    buf = (double*)arena.alloc(total * sizeof(double));
    std::vector<EwDesc> ds;
    ds.reserve(items.size());
    for (const Item& it : items) ds.push_back(ew_desc(EW_COPY, it.src, DT_F64, buf + it.off, DT_F64, (int64_t)it.n));
    rec.ew(std::move(ds));
  }
  // after the recorder ran: one transfer, then a wait
  void read(hipStream_t s) {
    host.assign(total, 0.0);
    if (total) dev::d2h(host.data(), buf, total * sizeof(double), s);
    dev::sync(s);
  }
  std::vector<double> slice(size_t off, size_t n) const {
    return std::vector<double>(host.begin() + off, host.begin() + off + n);
  }
};

inline RedDesc red_desc(const void* x, const void* y, int64_t n, double* out, int dt) {
  RedDesc r;
  std::memset(&r, 0, sizeof(r));
  r.x = x;
  r.y = y;
  r.n = n;
  r.out = out;
  r.dt = dt;
  return r;
}

inline QrDesc qr_desc(const double* A, int64_t sAr, int64_t sAc, double* Q, int64_t sQr, int64_t sQc, double* R,
               int64_t sRr, int64_t sRc, double* W, int m, int n) {
  QrDesc q;
  q.A = A;
  q.sAr = sAr;
  q.sAc = sAc;
  q.Q = Q;
  q.sQr = sQr;
  q.sQc = sQc;
  q.R = R;
  q.sRr = sRr;
  q.sRc = sRc;
  q.W = W;
  q.m = m;
  q.n = n;
  return q;
}


}  // namespace pe
