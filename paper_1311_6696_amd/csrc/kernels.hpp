// Device kernels of libpepsenv and their descriptor records.
//
// Every kernel is "grouped": one launch processes an array of independent
// descriptors (problems of any shapes), so that independent boundary rows,
// sandwiches, cluster windows and PEPS instances share launches.
#pragma once
#include "common.hpp"

namespace pe {

// ---------------------------------------------------------------------------
// Tensor contraction C[m,n] = alpha * sum_k A[m,k] B[k,n] + beta * C[m,n]
// where m, n and k are each a multi-index of up to 4 sub-dimensions with
// arbitrary strides in every operand (a GEMM over strided tensor views, so
// no permutation kernels are needed between the stages of a chain).
// ---------------------------------------------------------------------------
constexpr int TC_MAXD = 4;
struct TcDesc {
  const void* A;
  const void* B;
  void* C;
  int64_t sAm[TC_MAXD], sAk[TC_MAXD], sBk[TC_MAXD], sBn[TC_MAXD], sCm[TC_MAXD], sCn[TC_MAXD];
  int32_t dm[TC_MAXD], dn[TC_MAXD], dk[TC_MAXD];   // sub-dimension sizes, outermost first
  int32_t nm, nn, nk;                              // number of sub-dimensions (>= 1)
  int32_t M, N, K;
  int32_t tiles_n, tile_base;                      // filled when the op is recorded
  int32_t a_kfast, b_kfast;                        // global->LDS load order
  double alpha, beta;
  // Split-K (filled when the op is recorded): ksplit slices of kslice
  // elements each; slice s of tile t writes its partial tile, m fastest, to
  // part[(t*ksplit + s)*MT*NT]; a separate launch sums the slices in order.
  int32_t ksplit, kslice;
  double* part;
};

// Short, skinny FP64 contraction C[m][n] = alpha * sum_k A[m][k] B[k][n] with
// one stride per index (n <= 32, m and k of a few hundred to a few
// thousand): 32 x 32 output tiles, K in slices of TSK_KS, the slices of a
// tile summed in slice order by the last one to finish (no second launch).
constexpr int TSK_MT = 32, TSK_KS = 64;
struct TskDesc {
  const double* A;
  const double* B;
  double* C;
  int64_t sAm, sAk, sBk, sBn, sCm, sCn;
  int32_t M, N, K;
  int32_t ksplit;       // slices of TSK_KS
  int32_t tile_base;    // first workgroup: ceil(M / TSK_MT) * ksplit of them, slice fastest
  int32_t cnt_base;     // first arrival counter (one per row tile)
  double alpha;
  double* part;         // ceil(M / TSK_MT) * ksplit partial tiles of TSK_MT * 32 doubles
};
void launch_tsk(const TskDesc* d_desc, int n_desc, int n_blocks, unsigned* counters, hipStream_t s);

// Fused ket-bra contraction (one site's two layers applied in one launch):
//   Y[R; dr, gs] = sum_{p, q} (sum_{lu} X[R; lu, q] K[lu; dr, p]) B[p, q; gs]
// Each index group lists its sub-dimensions outermost first with their
// strides in the two tensors that hold it.
constexpr int KB_MAXD = 4;
struct KbGroup {
  int32_t n, size;
  int32_t dim[KB_MAXD];
  int64_t s0[KB_MAXD], s1[KB_MAXD];
};
struct KbDesc {
  const void* X;
  const void* K;
  const void* B;
  void* Y;
  KbGroup r;    // strides in X, Y (innermost unit-stride in both)
  KbGroup lu;   // X, K
  KbGroup q;    // X, B
  KbGroup p;    // K, B
  KbGroup dr;   // K, Y
  KbGroup gs;   // B, Y
  int32_t tile_base;   // first 16-row block of R, numbered across descriptors
};
// Launch of n_blocks 16-row blocks; nb1 = blocks of 16 over dr*p (1 or 2);
// lup = 4*ceil(max lu/4), pqp = 4*ceil(max p*q/4), qmax = max q.
void launch_kb(int prec, int out_dt, int nb1, const KbDesc* d_desc, int n_desc, int n_blocks, int lup, int pqp,
               int qmax, hipStream_t s);
int kb_lds_bytes(int prec, int nb1, int lup, int pqp, int qmax);
constexpr int KB_QC = 8;   // q values per shared-memory chunk

// Fused two-row column step (one column of the two-row sandwich): with every
// virtual leg of dimension 4 and physical dimension 2,
//   O[y; R,S,r,s; e] = sum L[x; L,M,l,m; a] T[a; u,v; e] K1[p; l,u,r,d] B1[p; m,v,s,g]
//                          K2[q; L,d,R,D] B2[q; M,g,S,G] Bb[x; D,G; y]
// (names of the left-to-right step; the right-to-left step is the same
// contraction with the horizontal roles exchanged through the strides).  One
// workgroup per output value e runs the whole chain for every x, all
// intermediates in LDS, accumulating over x in registers.  Site views list
// their strides as (physical, incoming leg, up, outgoing leg, down).
constexpr int K2_D = 4, K2_CHI = 32;   // leg dimension, largest bond
struct K2Desc {
  const double* L;
  const double* T;
  const double* B;
  double* O;
  const double* s[4];   // K1, B1, K2, B2
  int64_t sL[6];        // x, L, M, l, m, a
  int64_t sT[4];        // a, u, v, e
  int64_t sB[4];        // x, D, G, y
  int64_t sO[6];        // y, R, S, r, s, e
  int64_t ss[4][5];
  int32_t X, A, E, Y;   // bonds: x (L, Bb), a (L, T), e (T, O), y (Bb, O), each <= K2_CHI
  int32_t block_base;   // first workgroup of this descriptor (slice 0 of output value e = 0)
  // x slices per output value (filled when the op is recorded): with ns > 1
  // workgroup (sl, e) sums x over its slice only and writes the partial
  // result to part[(e*ns + sl)*K2_PART ...]; the last slice of e to finish
  // (arrival counter cnt_base + e) adds the ns partials in slice order and
  // stores O.  ns == 1: the workgroup stores O directly.
  int32_t ns;
  int32_t cnt_base, pad;
  double* part;
};
constexpr int K2_PART = K2_CHI / 4 * 1024;   // partial result of one (e, slice): 1024 threads x K2_CHI/4 values
// chmax: the largest bond (A or Y) of the launch's descriptors; counters:
// the arrival counters of the sliced descriptors (zero at launch).
void launch_k2(const K2Desc* d_desc, int n_desc, int n_blocks, int chmax, unsigned* counters, hipStream_t s);

// One-row chain step (D = 4, d = 2, float64), the ALS site step's and the
// one-row sandwich's first three contractions in one launch:
//   Y[x][d][g][r][s][e] = sum E[x][l][m][a] T[a][u][v][e] K[p][l][u][r][d] B[p][m][v][s][g]
// (a right-to-left step is the same with the roles of its horizontal legs
// exchanged through the strides).  One wave per (x, e), KC_W x per
// workgroup and pass; a workgroup makes xr passes over consecutive groups
// of x with the same e, reusing its staged sites and top boundary slab.
struct KcDesc {
  const double* E;
  const double* T;
  const double* s[2];   // ket K, bra B
  double* Y;
  int64_t sE[4];        // x, l, m, a
  int64_t sT[4];        // a, u, v, e
  int64_t ss[2][5];     // p, l, u, r, d  (bra: p, m, v, s, g)
  int64_t sY[6];        // x, d, g, r, s, e
  int32_t X, A, Ne;     // bonds x, a (<= K2_CHI) and e
  int32_t block_base;   // first workgroup of this descriptor: ceil(ceil(X / KC_W) / xr) * Ne of them, e fastest
  int32_t xr;           // groups of KC_W x values per workgroup (filled when the op is recorded)
  int32_t pad;
};
constexpr int KC_W = 8;   // waves (x values) per workgroup of the one-row chain step
void launch_kc(const KcDesc* d_desc, int n_desc, int n_blocks, hipStream_t s);

// Arithmetic of a contraction.
enum TcPrec : int { TP_F64 = 0, TP_F32 = 1, TP_BF16 = 2 };
// Tile shapes (MT x NT per 256-thread workgroup).
// TT_S16..TT_S80: the skinny kernel (64-row groups, N up to 16..80).
enum TcTile : int {
  TT_64x64 = 0, TT_128x32 = 1, TT_256x16 = 2, TT_32x128 = 3, TT_64x32 = 4, TT_64x16 = 5, TT_128x48 = 6, TT_64x80 = 7,
  TT_S16 = 8, TT_S32 = 9, TT_S48 = 10, TT_S64 = 11, TT_S80 = 12, TT_KB16 = 13, TT_KB32 = 14,
  TT_K2 = 15,   // the fused two-row column step (statistics slot only)
  TT_COUNT = 16
};
inline int tile_mt(int t) {
  static const int v[TT_COUNT] = {64, 128, 256, 32, 64, 64, 128, 64, 64, 64, 64, 64, 64, 16, 16, 256};
  return v[t];
}
inline int tile_nt(int t) {
  static const int v[TT_COUNT] = {64, 32, 16, 128, 32, 16, 48, 80, 16, 32, 48, 64, 80, 16, 32, 64};
  return v[t];
}
// Statistics slot of a contraction variant.
inline int tc_stat_index(int prec, int out_dt, int tile) { return (prec * 2 + out_dt) * TT_COUNT + tile; }

// out_dt: DT_F64 or DT_F32 (element type of C).  A and B are float64 for
// TP_F64 and float32 for TP_F32/TP_BF16.
void launch_tc(int prec, int out_dt, int tile, const TcDesc* d_desc, int n_desc, int n_tiles,
               hipStream_t s);
// Skinny contraction (N <= 16*nb, unit stride along m in A and C):
// descriptors' tile_base counts groups of 64 rows; kp = 4*ceil(max K/4) rows
// of B staged per descriptor; ksm in {8, 16} k-steps of A per load batch,
// nb in 1..5.
void launch_tcs(int prec, int out_dt, int nb, int ksm, const TcDesc* d_desc, int n_desc, int n_groups, int kp,
                hipStream_t s);
// Shared memory of one skinny workgroup (bytes).
int tcs_lds_bytes(int prec, int nb, int kp);
// Second half of a split-K contraction: C = alpha * (sum of the slices in
// slice order) + beta * C, one workgroup per output tile (n_tiles in all).
void launch_tc_reduce(int out_dt, int tile, const TcDesc* d_desc, int n_desc, int n_tiles, hipStream_t s);

// ---------------------------------------------------------------------------
// Householder QR of an m x n float64 matrix (m >= n), one workgroup each.
// Q (m x n, orthonormal columns) and optionally R (n x n) are written with
// arbitrary strides; the signs are fixed so that diag(R) >= 0.
// ---------------------------------------------------------------------------
struct QrDesc {
  const double* A;
  int64_t sAr, sAc;
  double* Q;
  int64_t sQr, sQc;
  double* R;        // may be null
  int64_t sRr, sRc;
  double* W;        // workspace of 2*m*n doubles
  int32_t m, n;
};
void launch_qr(const QrDesc* d_desc, int n_desc, hipStream_t s);
// Route for blocks up to m x n: a register-resident variant (>= 0), QR_CQ
// (CholeskyQR2 over several workgroups) or -1 (none fits), and the launch of
// a register-resident variant.
constexpr int QR_CQ = 1000;
int qr_variant_for(int m, int n);
void launch_qr_reg(int variant, const QrDesc* d_desc, int n_desc, hipStream_t s);

// CholeskyQR2 of a tall block (m <= 512, n <= 32) over ceil(m / CQ_ROWS)
// workgroups that wait for each other's factors: one launch, all of whose
// workgroups (at most CQ_MAXWG) must be resident at once.
constexpr int CQ_ROWS = 128;
constexpr int CQ_MAXP = 4;       // workgroups per block (m <= CQ_ROWS * CQ_MAXP)
constexpr int CQ_MAXWG = 256;    // workgroups per launch: one per compute unit
struct CqDesc {
  QrDesc q;             // the block (q.W unused)
  double* ws;           // cq_ws_doubles(m, n) doubles, private to this block during the launch
  int32_t cnt;          // its arrival counter: an index into the launch's counters, zero at launch
  int32_t P;            // workgroups of the block
  int32_t block_base;   // its first workgroup in the launch
  int32_t pad;
};
size_t cq_ws_doubles(int m, int n);
// nb: 16-column blocks of the widest block (1 or 2); n_blocks: workgroups.
void launch_cq(int nb, const CqDesc* d_desc, int n_desc, int n_blocks, unsigned* counters, hipStream_t s);
// Zero n counters (a kernel, so that it can sit in a captured graph).
void launch_cq_clear(unsigned* counters, int n, hipStream_t s);

// ---------------------------------------------------------------------------
// Deterministic sums: out = sum_i x_i * y_i (y null -> sum x_i^2), in two
// passes over fixed partitions (bitwise reproducible).
// ---------------------------------------------------------------------------
struct RedDesc {
  const void* x;
  const void* y;
  int64_t n;
  double* out;
  int32_t dt;          // element type of x and y
  int32_t block_base;  // first block of this descriptor (filled on record)
  int32_t nblocks;
  int32_t part_base;   // offset into the partial-sum buffer
};
void launch_reduce(const RedDesc* d_desc, int n_desc, int n_blocks, double* partials, hipStream_t s);

// ---------------------------------------------------------------------------
// Elementwise operations on contiguous buffers.
// ---------------------------------------------------------------------------
enum EwKind : int {
  EW_COPY = 0,        // dst = src (with type conversion)
  EW_PHYS = 1,        // dst[p*L+i] = sum_q op[p][q] src[q*L+i]   (2x2 operator, L = n/2)
  EW_FILL = 2,        // dst = a
  EW_SPLITMIX = 3,    // dst[i] = SplitMix64 value i of stream state `key`, in [-1, 1)
  EW_RSQRT = 4,       // dst = src / sqrt(*sptr)
  EW_IDENTITY = 5,    // dst = a * identity (n = D*D)
  EW_NONFINITE = 6,   // dst[0] = a wherever src holds NaN or Inf (dst untouched otherwise)
  EW_LOGACC = 7,      // one thread: dst[0] = 0, dst[k+1] = dst[k] + log(*src[k]) / 2 for k < n
                      //   (src: device array of n pointers to squared norms)
};
struct EwDesc {
  const void* src;
  void* dst;
  int64_t n;
  int32_t src_dt, dst_dt;
  int32_t kind;
  int32_t block_base;
  int32_t nblocks;
  int32_t dim;          // matrix dimension for EW_IDENTITY
  double a;
  double op[4];
  uint64_t key;
  const double* sptr;
};
void launch_ew(const EwDesc* d_desc, int n_desc, int n_blocks, hipStream_t s);

// ---------------------------------------------------------------------------
// CU_0 separable boundaries (D' = 1): for one lattice direction, the rows of
// the frame are absorbed one after another; each absorption is an ALS over
// the row's sites whose local solution is sigma_c = b_c / |b_c| (the norm
// matrix is a multiple of the identity), sweeping left-right-left until no
// sigma changes by more than `tol` or `max_sweeps` sweeps have run.  One
// workgroup per descriptor; virtual bond dimensions up to SEP_MAXD.
// ---------------------------------------------------------------------------
constexpr int SEP_MAXD = 8;
struct SepSite {
  const double* A;
  int32_t d, Dl, Du, Dr, Dd, pad;
  int64_t sp, sl, su, sr, sd;   // strides of the frame's (p, l, u, r, d) legs
};
struct SepDesc {
  int32_t Lr, Lc, max_sweeps;
  int32_t dmax;           // largest virtual bond of the direction's sites
  double tol;
  const SepSite* sites;   // Lr*Lc, frame row-major
  double* sig;            // sigma of frame row k, column c at sig + off[k*Lc + c] (Dd x Dd)
  const int64_t* off;
  double* work;           // (3*Lc + 3) * SEP_MAXD^2 + 2 * SEP_MAXD^4 doubles
  int32_t* sweeps;        // Lr-1 entries
  double* delta;          // Lr-1 entries
};
// dmax: the largest dmax of the descriptors (every leg is padded to it);
// the physical dimension must be at most 2.
void launch_sep(const SepDesc* d_desc, int n_desc, int dmax, hipStream_t s);

// SplitMix64 (Steele, Lea, Flood 2014): output function and stream state.
__host__ __device__ inline uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t SPLITMIX_GAMMA = 0x9E3779B97F4A7C15ull;

}  // namespace pe
