// Device kernels of libpepsenv (gfx950 / CDNA4).
#include <algorithm>
#include <climits>
#include <type_traits>

#include "kernels.hpp"

namespace pe {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

// DPP move of a double (both 32-bit halves); lanes without a source read 0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ inline double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, ROW_MASK, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wave, returned to every lane.  Inclusive scan
// inside each 16-lane row by row_shr 1,2,4,8, then row_bcast:15 and
// row_bcast:31 carry the row totals so that lane 63 holds the sum.  The
// summation order is fixed, so every lane gets the same bits.
__device__ inline double wave_sum(double v) {
  v += dpp_d<0x111>(v);        // row_shr:1
  v += dpp_d<0x112>(v);        // row_shr:2
  v += dpp_d<0x114>(v);        // row_shr:4
  v += dpp_d<0x118>(v);        // row_shr:8
  v += dpp_d<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Value of lane l (uniform) of a double, returned to every lane.
__device__ inline double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 256 threads of a workgroup; every thread receives the same value.
__device__ inline double block_sum256(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return s;
}

// ===========================================================================
// Tensor contraction on MFMA.  The 16x16 MFMA tile is issued as D = B^T A^T
// so that lane bits 0..3 index m: stores are then contiguous along m, which
// is the unit-stride index of every large intermediate of the chains.
// Accumulator element r of lane l holds (m = l & 15, n = row(l, r)).
// ===========================================================================
struct PolF64 {
  using T = double;
  using L = double;
  using F = double;
  using Acc = d4_t;
  static constexpr int KT = 16, KS = 4;
  __device__ static inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
  template <int LD>
  __device__ static inline F frag(const L (*X)[LD], int ks, int cb, int lane) {
    return X[ks * 4 + (lane >> 4)][cb + (lane & 15)];
  }
  __device__ static inline Acc mma(F b, F a, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c, 0, 0, 0);
  }
};

struct PolF32 {
  using T = float;
  using L = float;
  using F = float;
  using Acc = f4_t;
  static constexpr int KT = 16, KS = 4;
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
  template <int LD>
  __device__ static inline F frag(const L (*X)[LD], int ks, int cb, int lane) {
    return X[ks * 4 + (lane >> 4)][cb + (lane & 15)];
  }
  __device__ static inline Acc mma(F b, F a, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(b, a, c, 0, 0, 0);
  }
};

struct PolBF16 {
  using T = float;   // operands are stored as float32 and rounded to bf16 (RNE) on the way to LDS
  using L = __bf16;
  using F = bf8_t;
  using Acc = f4_t;
  static constexpr int KT = 32, KS = 32;
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
  template <int LD>
  __device__ static inline F frag(const L (*X)[LD], int ks, int cb, int lane) {
    F f;
    const int k0 = ks * 32 + 8 * (lane >> 4), c = cb + (lane & 15);
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = X[k0 + e][c];
    return f;
  }
  __device__ static inline Acc mma(F b, F a, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, a, c, 0, 0, 0);
  }
};

// Shared-memory staging of one workgroup of tc_kernel.
// k offsets are kept for a window of TC_KWIN consecutive k values (one
// index decomposition per thread), refreshed every TC_KWIN / KT chunks.
constexpr int TC_KWIN = 256;

template <class L, int MT, int NT, int KT>
struct TcSmem {
  L As[KT][MT + 2];
  L Bs[KT][NT + 2];
  int64_t oAm[MT], oCm[MT], oBn[NT], oCn[NT], oAk[TC_KWIN], oBk[TC_KWIN];
};

// One output tile (or one K-slice of it) of descriptor d; `wg` numbers the
// tile's workgroup slot inside the descriptor.
template <class P, class TC, int MT, int NT, int WM, int WN>
__device__ inline void tc_tile(const TcDesc& d, int wg, TcSmem<typename P::L, MT, NT, P::KT>& sm) {
  using T = typename P::T;
  using L = typename P::L;
  constexpr int KT = P::KT;
  constexpr int WTM = MT / WM, WTN = NT / WN, MB = WTM / 16, NB = WTN / 16;
  constexpr int EA = MT * KT / 256, EB = NT * KT / 256;
  static_assert(EA >= 1 && EB >= 1 && MB >= 1 && NB >= 1, "tile");
  static_assert(EA * 256 == MT * KT && EB * 256 == NT * KT, "a chunk is a whole number of loads per thread");
  auto& As = sm.As;
  auto& Bs = sm.Bs;
  int64_t* oAm = sm.oAm;
  int64_t* oCm = sm.oCm;
  int64_t* oBn = sm.oBn;
  int64_t* oCn = sm.oCn;
  int64_t* oAk = sm.oAk;
  int64_t* oBk = sm.oBk;

  // The empty asm hides the thread index from loop-invariant hoisting across
  // the tile loop: hoisted per-thread addresses would stay live in VGPRs
  // for the whole walk and cost a wave of occupancy.
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int M = d.M, N = d.N;
  const int ksplit = d.ksplit;
  const int t = wg / ksplit, slice = wg - t * ksplit;
  const int m0 = (t / d.tiles_n) * MT, n0 = (t % d.tiles_n) * NT;
  const int kbeg = slice * d.kslice;
  const int K = min(d.K, kbeg + d.kslice);   // this slice covers [kbeg, K)
  const T* __restrict__ A = (const T*)d.A;
  const T* __restrict__ B = (const T*)d.B;
  TC* __restrict__ C = (TC*)d.C;
  const int a_kfast = d.a_kfast, b_kfast = d.b_kfast;

  static_assert(TC_KWIN % KT == 0 && TC_KWIN <= 256, "whole chunks per k window, one entry per thread");
  // m and n offsets: one decomposition per row or column, spread over the
  // workgroup (m rows on the first MT threads, n columns after them)
  for (int i = tid; i < MT + NT; i += 256) {
    int64_t o1 = 0, o2 = 0;
    if (i < MT) {
      int m = m0 + i;
      if (m < M)
        for (int j = d.nm - 1; j >= 0; --j) {
          const int dj = d.dm[j];
          const int x = m % dj;
          m /= dj;
          o1 += (int64_t)x * d.sAm[j];
          o2 += (int64_t)x * d.sCm[j];
        }
      oAm[i] = o1;
      oCm[i] = o2;
    } else {
      int n = n0 + i - MT;
      if (n < N)
        for (int j = d.nn - 1; j >= 0; --j) {
          const int dj = d.dn[j];
          const int x = n % dj;
          n /= dj;
          o1 += (int64_t)x * d.sBn[j];
          o2 += (int64_t)x * d.sCn[j];
        }
      oBn[i - MT] = o1;
      oCn[i - MT] = o2;
    }
  }
  // k offsets of the window starting at chunk c0
  constexpr int CPW = TC_KWIN / KT;
  auto k_window = [&](int c0) {
    int k = kbeg + c0 * KT + tid;
    int64_t oa = 0, ob = 0;
    if (k < K)
      for (int j = d.nk - 1; j >= 0; --j) {
        const int dj = d.dk[j];
        const int x = k % dj;
        k /= dj;
        oa += (int64_t)x * d.sAk[j];
        ob += (int64_t)x * d.sBk[j];
      }
    oAk[tid] = oa;
    oBk[tid] = ob;
  };
  k_window(0);
  __syncthreads();

  T ra[EA], rb[EB];
  // Element e of a thread covers linear index tid + 256*e of the KT x MT (or
  // KT x NT) chunk, fastest along k when that is the operand's unit stride.
  auto a_at = [&](int e, int& mm, int& kk) {
    const int idx = tid + 256 * e;
    if (a_kfast) { kk = idx % KT; mm = idx / KT; }
    else { mm = idx % MT; kk = idx / MT; }
  };
  auto b_at = [&](int e, int& nn, int& kk) {
    const int idx = tid + 256 * e;
    if (b_kfast) { kk = idx % KT; nn = idx / KT; }
    else { nn = idx % NT; kk = idx / NT; }
  };
  auto load = [&](int kc) {
    const int k0 = kbeg + kc * KT, w0 = (kc % CPW) * KT;   // chunk kc's place in its k window
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int mm, kk;
      a_at(e, mm, kk);
      const bool ok = (m0 + mm < M) && (k0 + kk < K);
      ra[e] = ok ? A[oAm[mm] + oAk[w0 + kk]] : T(0);
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int nn, kk;
      b_at(e, nn, kk);
      const bool ok = (n0 + nn < N) && (k0 + kk < K);
      rb[e] = ok ? B[oBn[nn] + oBk[w0 + kk]] : T(0);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int mm, kk;
      a_at(e, mm, kk);
      As[kk][mm] = (L)ra[e];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int nn, kk;
      b_at(e, nn, kk);
      Bs[kk][nn] = (L)rb[e];
    }
  };

  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave % WM, wn = wave / WM;
  typename P::Acc acc[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  const int nchunks = (K - kbeg + KT - 1) / KT;
  load(0);
  for (int kc = 0; kc < nchunks; ++kc) {
    __syncthreads();
    store();
    if (kc + 1 < nchunks && (kc + 1) % CPW == 0) k_window(kc + 1);   // the last chunk's offsets are read
    __syncthreads();
    if (kc + 1 < nchunks) load(kc + 1);
    // Every k step of the chunk runs (those past K multiply the zeros staged
    // for them): a branch between the MFMAs would make the compiler move the
    // accumulators out of and back into the matrix registers around it.
#pragma unroll
    for (int ks = 0; ks < KT / P::KS; ++ks) {
      typename P::F af[MB], bf[NB];
#pragma unroll
      for (int i = 0; i < MB; ++i) af[i] = P::template frag<MT + 2>(As, ks, wm * WTM + i * 16, lane);
#pragma unroll
      for (int j = 0; j < NB; ++j) bf[j] = P::template frag<NT + 2>(Bs, ks, wn * WTN + j * 16, lane);
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = P::mma(bf[j], af[i], acc[i][j]);
    }
  }

  const double alpha = d.alpha, beta = d.beta;
  if (ksplit == 1) {
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ml = wm * WTM + i * 16 + (lane & 15);
          const int nl = wn * WTN + j * 16 + P::row(lane, r);
          if (m0 + ml < M && n0 + nl < N) {
            const int64_t off = oCm[ml] + oCn[nl];
            double v = alpha * (double)acc[i][j][r];
            if (beta != 0.0) v += beta * (double)C[off];
            C[off] = (TC)v;
          }
        }
    return;
  }
  // split-K: this slice's partial tile, m fastest (coalesced for the
  // reduction, whose stores run along m)
  double* __restrict__ part = d.part + ((int64_t)t * ksplit + slice) * (MT * NT);
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ml = wm * WTM + i * 16 + (lane & 15);
        const int nl = wn * WTN + j * 16 + P::row(lane, r);
        part[nl * MT + ml] = (double)acc[i][j][r];
      }
}

// Grouped contraction: workgroup slots are numbered consecutively across
// the descriptors (tile_base); each workgroup walks the slots bid,
// bid + gridDim.x, ... so that large launches run a resident grid.  The
// owning descriptor only moves forward along that walk.
template <class P, class TC, int MT, int NT, int WM, int WN>
__global__ __launch_bounds__(256) void tc_kernel(const TcDesc* __restrict__ ds, int nd, int nslots) {
  __shared__ TcSmem<typename P::L, MT, NT, P::KT> sm;
  int lo = 0;
  for (int bid = blockIdx.x; bid < nslots; bid += gridDim.x) {
    if (lo + 1 < nd && ds[lo + 1].tile_base <= bid) {
      int a = lo + 1, b = nd - 1;
      while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (ds[mid].tile_base <= bid) a = mid; else b = mid - 1;
      }
      lo = a;
    }
    tc_tile<P, TC, MT, NT, WM, WN>(ds[lo], bid - ds[lo].tile_base, sm);
    __syncthreads();   // shared offsets and staging are rewritten by the next slot
  }
}

// Resident workgroups per launch for large groups: 256 CUs, several
// workgroups of 256 threads each.
constexpr int TC_GRID_CAP = 256 * 8;

template <class P, class TC>
static void launch_tc_tile(int tile, const TcDesc* d, int nd, int nt, hipStream_t s) {
  const int g = nt < TC_GRID_CAP ? nt : TC_GRID_CAP;
  switch (tile) {
    case TT_64x64: tc_kernel<P, TC, 64, 64, 2, 2><<<g, 256, 0, s>>>(d, nd, nt); break;
    case TT_128x32: tc_kernel<P, TC, 128, 32, 4, 1><<<g, 256, 0, s>>>(d, nd, nt); break;
    case TT_256x16: tc_kernel<P, TC, 256, 16, 4, 1><<<g, 256, 0, s>>>(d, nd, nt); break;
    case TT_32x128: tc_kernel<P, TC, 32, 128, 1, 4><<<g, 256, 0, s>>>(d, nd, nt); break;
    case TT_64x32: tc_kernel<P, TC, 64, 32, 2, 2><<<g, 256, 0, s>>>(d, nd, nt); break;
    case TT_64x16: tc_kernel<P, TC, 64, 16, 4, 1><<<g, 256, 0, s>>>(d, nd, nt); break;
    case TT_128x48: tc_kernel<P, TC, 128, 48, 4, 1><<<g, 256, 0, s>>>(d, nd, nt); break;
    case TT_64x80: tc_kernel<P, TC, 64, 80, 4, 1><<<g, 256, 0, s>>>(d, nd, nt); break;
    default: throw Error(ST_INVALID, "bad tile");
  }
}

void launch_tc(int prec, int out_dt, int tile, const TcDesc* d, int nd, int nt, hipStream_t s) {
  if (nt <= 0) return;
  if (prec == TP_F64) {
    if (out_dt != DT_F64) throw Error(ST_INVALID, "f64 contraction writes f64");
    launch_tc_tile<PolF64, double>(tile, d, nd, nt, s);
  } else if (prec == TP_F32) {
    if (out_dt == DT_F64) launch_tc_tile<PolF32, double>(tile, d, nd, nt, s);
    else launch_tc_tile<PolF32, float>(tile, d, nd, nt, s);
  } else {
    if (out_dt == DT_F64) launch_tc_tile<PolBF16, double>(tile, d, nd, nt, s);
    else launch_tc_tile<PolBF16, float>(tile, d, nd, nt, s);
  }
  PE_HIP(hipGetLastError());
}

// ===========================================================================
// Skinny contraction: small K and N (<= 16*NB), long M with unit stride in
// A and C.  Each wave owns a 16-row strip and reads its A fragments straight
// from global memory into registers, KSM k-steps at a time (no
// shared-memory staging, no barriers inside a descriptor), so a wave keeps
// up to KSM loads in flight.  B and the k/n offset tables are
// staged in shared memory once per descriptor.  Slots are groups of four
// strips (64 rows), numbered across descriptors by tile_base.
// ===========================================================================
__host__ __device__ constexpr int tcs_bpad(int nb) { return 16 * nb + 2; }

// Offsets of every k < kp (in A and in B) and every n < np (in B and in C)
// of a descriptor: one mixed-radix decomposition per entry, the k and n
// entries spread over the workgroup's threads.  Entries past K or N are 0.
__device__ inline void tc_index_tables(const TcDesc& d, int kp, int np, int64_t* oAk, int64_t* oBk, int64_t* oBn,
                                       int64_t* oCn, int tid) {
  for (int i = tid; i < kp + np; i += 256) {
    int64_t o1 = 0, o2 = 0;
    if (i < kp) {
      int k = i;
      if (k < d.K)
        for (int j = d.nk - 1; j >= 0; --j) {
          const int x = k % d.dk[j];
          k /= d.dk[j];
          o1 += (int64_t)x * d.sAk[j];
          o2 += (int64_t)x * d.sBk[j];
        }
      oAk[i] = o1;
      oBk[i] = o2;
    } else {
      int n = i - kp;
      if (n < d.N)
        for (int j = d.nn - 1; j >= 0; --j) {
          const int x = n % d.dn[j];
          n /= d.dn[j];
          o1 += (int64_t)x * d.sBn[j];
          o2 += (int64_t)x * d.sCn[j];
        }
      oBn[i - kp] = o1;
      oCn[i - kp] = o2;
    }
  }
}

template <class P, class TC, int NB, int KSM>
__global__ __launch_bounds__(256) void tcs_kernel(const TcDesc* __restrict__ ds, int nd, int ngroups, int kp) {
  using T = typename P::T;
  using L = typename P::L;
  static_assert(P::KS == 4, "fragments of four k per lane group");
  constexpr int NP = 16 * NB, NPAD = tcs_bpad(NB);
  extern __shared__ __align__(16) unsigned char tcs_smem[];
  L* Bs = (L*)tcs_smem;                                                      // [kp][NPAD]
  int64_t* oAk = (int64_t*)(tcs_smem + ((size_t)kp * NPAD * sizeof(L) + 15) / 16 * 16);   // [kp]
  int64_t* oBk = oAk + kp;                                                   // [kp]
  int64_t* oCn = oBk + kp;                                                   // [NP]
  int64_t* oBn = oCn + NP;                                                   // [NP]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // contiguous blocks of groups per workgroup: a workgroup crosses few
  // descriptor boundaries, so B is staged rarely
  const int per = (ngroups + gridDim.x - 1) / gridDim.x;
  const int gend = min(ngroups, (blockIdx.x + 1) * per);
  int cur = -1;
  for (int g = blockIdx.x * per; g < gend; ++g) {
    int lo = cur;
    if (cur < 0 || (cur + 1 < nd && ds[cur + 1].tile_base <= g)) {
      int a = cur < 0 ? 0 : cur + 1, b = nd - 1;
      while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (ds[mid].tile_base <= g) a = mid; else b = mid - 1;
      }
      lo = a;
    }
    const TcDesc& d = ds[lo];
    const int M = d.M, N = d.N, K = d.K;
    if (lo != cur) {
      __syncthreads();   // the previous descriptor's tables are no longer read
      tc_index_tables(d, kp, NP, oAk, oBk, oBn, oCn, tid);
      __syncthreads();
      const T* __restrict__ B = (const T*)d.B;
      for (int i = tid; i < kp * NP; i += 256) {
        const int k = i / NP, n = i - k * NP;
        Bs[k * NPAD + n] = (L)((k < K && n < N) ? B[oBk[k] + oBn[n]] : T(0));
      }
      __syncthreads();
      cur = lo;
    }
    const int m = ((g - d.tile_base) * 4 + wave) * 16 + (lane & 15);
    const bool mok = m < M;
    int64_t oa = 0, oc = 0;
    if (mok) {
      int mm = m;
      for (int j = d.nm - 1; j >= 0; --j) {
        const int x = mm % d.dm[j];
        mm /= d.dm[j];
        oa += (int64_t)x * d.sAm[j];
        oc += (int64_t)x * d.sCm[j];
      }
    }
    const T* __restrict__ A = (const T*)d.A;
    const int nks = (K + 3) >> 2;
    typename P::Acc acc[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[j][r] = 0;
    // K in blocks of KSM k-steps: all fragment loads of a block are issued
    // before its first MFMA
    for (int kb = 0; kb < nks; kb += KSM) {
      T af[KSM];
#pragma unroll
      for (int q = 0; q < KSM; ++q) {
        const int k = 4 * (kb + q) + (lane >> 4);
        af[q] = (kb + q < nks && mok && k < K) ? A[oa + oAk[k]] : T(0);
      }
#pragma unroll
      for (int q = 0; q < KSM; ++q) {
        if (kb + q >= nks) break;
        const L* brow = Bs + (4 * (kb + q) + (lane >> 4)) * NPAD + (lane & 15);
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[j] = P::mma(brow[16 * j], (typename P::F)af[q], acc[j]);
      }
    }
    TC* __restrict__ C = (TC*)d.C;
    const double alpha = d.alpha, beta = d.beta;
    if (mok) {
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int n = 16 * j + P::row(lane, r);
          if (n < N) {
            const int64_t off = oc + oCn[n];
            double v = alpha * (double)acc[j][r];
            if (beta != 0.0) v += beta * (double)C[off];
            C[off] = (TC)v;
          }
        }
    }
  }
}

// BF16 form of the skinny contraction: fragments of eight consecutive k per
// lane (16x16x32 MFMA), A read as float32 and rounded to bf16 (RNE) in
// registers, B staged once per descriptor as bf16 with k contiguous so a
// fragment is one 16-byte shared-memory read.  Same accumulation order as
// the tiled bf16 kernel.
template <class TC, int NB, int KSM>
__global__ __launch_bounds__(256) void tcs_bf16_kernel(const TcDesc* __restrict__ ds, int nd, int ngroups, int kp) {
  constexpr int NP = 16 * NB;
  const int kpad = kp + 8;
  extern __shared__ __align__(16) unsigned char tcs_smem[];
  __bf16* Bs = (__bf16*)tcs_smem;                                                       // [NP][kpad]
  int64_t* oAk = (int64_t*)(tcs_smem + ((size_t)NP * kpad * sizeof(__bf16) + 15) / 16 * 16);   // [kp]
  int64_t* oBk = oAk + kp;                                                              // [kp]
  int64_t* oCn = oBk + kp;                                                              // [NP]
  int64_t* oBn = oCn + NP;                                                              // [NP]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (ngroups + gridDim.x - 1) / gridDim.x;
  const int gend = min(ngroups, (blockIdx.x + 1) * per);
  int cur = -1;
  for (int g = blockIdx.x * per; g < gend; ++g) {
    int lo = cur;
    if (cur < 0 || (cur + 1 < nd && ds[cur + 1].tile_base <= g)) {
      int a = cur < 0 ? 0 : cur + 1, b = nd - 1;
      while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (ds[mid].tile_base <= g) a = mid; else b = mid - 1;
      }
      lo = a;
    }
    const TcDesc& d = ds[lo];
    const int M = d.M, N = d.N, K = d.K;
    if (lo != cur) {
      __syncthreads();
      tc_index_tables(d, kp, NP, oAk, oBk, oBn, oCn, tid);
      __syncthreads();
      const float* __restrict__ B = (const float*)d.B;
      for (int i = tid; i < kp * NP; i += 256) {
        const int k = i / NP, n = i - k * NP;
        Bs[n * kpad + k] = (__bf16)((k < K && n < N) ? B[oBk[k] + oBn[n]] : 0.f);
      }
      __syncthreads();
      cur = lo;
    }
    const int m = ((g - d.tile_base) * 4 + wave) * 16 + (lane & 15);
    const bool mok = m < M;
    int64_t oa = 0, oc = 0;
    if (mok) {
      int mm = m;
      for (int j = d.nm - 1; j >= 0; --j) {
        const int x = mm % d.dm[j];
        mm /= d.dm[j];
        oa += (int64_t)x * d.sAm[j];
        oc += (int64_t)x * d.sCm[j];
      }
    }
    const float* __restrict__ A = (const float*)d.A;
    const int nks = (K + 31) >> 5;
    f4_t acc[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[j][r] = 0.f;
    const int k8 = 8 * (lane >> 4);
    for (int kb = 0; kb < nks; kb += KSM) {
      float af[KSM][8];
#pragma unroll
      for (int q = 0; q < KSM; ++q)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = 32 * (kb + q) + k8 + e;
          af[q][e] = (kb + q < nks && mok && k < K) ? A[oa + oAk[k]] : 0.f;
        }
#pragma unroll
      for (int q = 0; q < KSM; ++q) {
        if (kb + q >= nks) break;
        bf8_t a8;
#pragma unroll
        for (int e = 0; e < 8; ++e) a8[e] = (__bf16)af[q][e];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const bf8_t b8 = *(const bf8_t*)(Bs + (16 * j + (lane & 15)) * kpad + 32 * (kb + q) + k8);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b8, a8, acc[j], 0, 0, 0);
        }
      }
    }
    TC* __restrict__ C = (TC*)d.C;
    const double alpha = d.alpha, beta = d.beta;
    if (mok) {
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int n = 16 * j + 4 * (lane >> 4) + r;
          if (n < N) {
            const int64_t off = oc + oCn[n];
            double v = alpha * (double)acc[j][r];
            if (beta != 0.0) v += beta * (double)C[off];
            C[off] = (TC)v;
          }
        }
    }
  }
}

int tcs_lds_bytes(int prec, int nb, int kp) {
  const size_t tables = (size_t)2 * (kp + 16 * nb) * sizeof(int64_t);   // oAk, oBk, oCn, oBn
  if (prec == TP_BF16) return (int)(((size_t)16 * nb * (kp + 8) * 2 + 15) / 16 * 16 + tables);
  const size_t el = prec == TP_F64 ? sizeof(double) : sizeof(float);
  return (int)(((size_t)kp * tcs_bpad(nb) * el + 15) / 16 * 16 + tables);
}

// One resident wave of workgroups (occupancy x compute units), so the
// contiguous group ranges finish together.
template <class K>
static int resident_grid(K kernel, int lds, int want) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    PE_HIP(hipGetDevice(&dev));
    PE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  }
  int occ = 0;
  PE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, 256, lds));
  const int cap = std::max(1, occ) * cus;
  return want < cap ? want : cap;
}

template <class P, class TC, int NB>
static void launch_tcs_nb(int ksm, const TcDesc* d, int nd, int ngroups, int kp, hipStream_t s) {
  const int lds = tcs_lds_bytes(std::is_same<typename P::T, double>::value ? TP_F64 : TP_F32, NB, kp);
  switch (ksm) {
    case 8: {
      const int g = resident_grid(tcs_kernel<P, TC, NB, 8>, lds, ngroups);
      tcs_kernel<P, TC, NB, 8><<<g, 256, lds, s>>>(d, nd, ngroups, kp);
      break;
    }
    case 16: {
      const int g = resident_grid(tcs_kernel<P, TC, NB, 16>, lds, ngroups);
      tcs_kernel<P, TC, NB, 16><<<g, 256, lds, s>>>(d, nd, ngroups, kp);
      break;
    }
    default: throw Error(ST_INVALID, "bad skinny k range");
  }
}

template <class TC, int NB>
static void launch_tcs_bf16_nb(int ksm, const TcDesc* d, int nd, int ngroups, int kp, hipStream_t s) {
  const int lds = tcs_lds_bytes(TP_BF16, NB, kp);
  switch (ksm) {
    case 2: {
      const int g = resident_grid(tcs_bf16_kernel<TC, NB, 2>, lds, ngroups);
      tcs_bf16_kernel<TC, NB, 2><<<g, 256, lds, s>>>(d, nd, ngroups, kp);
      break;
    }
    case 4: {
      const int g = resident_grid(tcs_bf16_kernel<TC, NB, 4>, lds, ngroups);
      tcs_bf16_kernel<TC, NB, 4><<<g, 256, lds, s>>>(d, nd, ngroups, kp);
      break;
    }
    default: throw Error(ST_INVALID, "bad skinny k range");
  }
}

template <class TC>
static void launch_tcs_bf16(int nb, int ksm, const TcDesc* d, int nd, int ngroups, int kp, hipStream_t s) {
  switch (nb) {
    case 1: launch_tcs_bf16_nb<TC, 1>(ksm, d, nd, ngroups, kp, s); break;
    case 2: launch_tcs_bf16_nb<TC, 2>(ksm, d, nd, ngroups, kp, s); break;
    case 3: launch_tcs_bf16_nb<TC, 3>(ksm, d, nd, ngroups, kp, s); break;
    case 4: launch_tcs_bf16_nb<TC, 4>(ksm, d, nd, ngroups, kp, s); break;
    case 5: launch_tcs_bf16_nb<TC, 5>(ksm, d, nd, ngroups, kp, s); break;
    default: throw Error(ST_INVALID, "bad skinny width");
  }
}

template <class P, class TC>
static void launch_tcs_p(int nb, int ksm, const TcDesc* d, int nd, int ngroups, int kp, hipStream_t s) {
  switch (nb) {
    case 1: launch_tcs_nb<P, TC, 1>(ksm, d, nd, ngroups, kp, s); break;
    case 2: launch_tcs_nb<P, TC, 2>(ksm, d, nd, ngroups, kp, s); break;
    case 3: launch_tcs_nb<P, TC, 3>(ksm, d, nd, ngroups, kp, s); break;
    case 4: launch_tcs_nb<P, TC, 4>(ksm, d, nd, ngroups, kp, s); break;
    case 5: launch_tcs_nb<P, TC, 5>(ksm, d, nd, ngroups, kp, s); break;
    default: throw Error(ST_INVALID, "bad skinny width");
  }
}

void launch_tcs(int prec, int out_dt, int nb, int ksm, const TcDesc* d, int nd, int ngroups, int kp, hipStream_t s) {
  if (ngroups <= 0) return;
  if (kp < 4 || kp % 4 != 0) throw Error(ST_INVALID, "bad skinny k range");
  if (prec == TP_F64) {
    if (out_dt != DT_F64) throw Error(ST_INVALID, "f64 contraction writes f64");
    launch_tcs_p<PolF64, double>(nb, ksm, d, nd, ngroups, kp, s);
  } else if (prec == TP_F32) {
    if (out_dt == DT_F64) launch_tcs_p<PolF32, double>(nb, ksm, d, nd, ngroups, kp, s);
    else launch_tcs_p<PolF32, float>(nb, ksm, d, nd, ngroups, kp, s);
  } else {
    if (kp % 32 != 0) throw Error(ST_INVALID, "bad skinny k range");
    if (out_dt == DT_F64) launch_tcs_bf16<double>(nb, ksm, d, nd, ngroups, kp, s);
    else launch_tcs_bf16<float>(nb, ksm, d, nd, ngroups, kp, s);
  }
  PE_HIP(hipGetLastError());
}

// ===========================================================================
// Fused ket-bra contraction (see KbDesc).  One workgroup per 16-row block of
// R at a time.  Phase 1: for a chunk of KB_QC values of q, waves form
// Z_q[R][dr,p] = X[R; lu, q] K[lu; dr, p] on MFMA (A fragments straight from
// global memory, K staged in shared memory) and leave Z in shared memory.
// Phase 2: waves accumulate Y[R; dr, gs] += Z[R; dr, (p, q)] B[(p, q); gs]
// for their dr values.  The ket intermediate never reaches global memory.
// Limits of this kernel: dr*p <= 16*NB1, p <= 2, gs <= 16, dr <= 16, lu <= 64.
// ===========================================================================
__device__ inline int64_t kb_off(const KbGroup& g, int v, bool second) {
  int64_t o = 0;
  for (int j = g.n - 1; j >= 0; --j) {
    const int x = v % g.dim[j];
    v /= g.dim[j];
    o += (int64_t)x * (second ? g.s1[j] : g.s0[j]);
  }
  return o;
}

__host__ __device__ constexpr int kb_np1pad(int nb1) { return 16 * nb1 + 2; }

template <class P, class TC, int NB1, int KS1>
__global__ __launch_bounds__(256) void kb_kernel(const KbDesc* __restrict__ ds, int nd, int nblocks, int lup,
                                                 int pqp, int qmax) {
  using T = typename P::T;
  using L = typename P::L;
  static_assert(P::KS == 4, "fragments of four k per lane group");
  constexpr int NP1 = 16 * NB1, NP1PAD = kb_np1pad(NB1), BPAD = 18, DRW = 4, QPW = KB_QC / 4;
  extern __shared__ __align__(16) unsigned char kb_smem[];
  L* Ks = (L*)kb_smem;                               // [lup][NP1PAD]
  L* Bs = Ks + (size_t)lup * NP1PAD;                 // [pqp][BPAD]
  L* Zs = Bs + (size_t)pqp * BPAD;                   // [KB_QC][NP1][16]
  int64_t* oXlu = (int64_t*)(kb_smem + (((size_t)lup * NP1PAD + (size_t)pqp * BPAD + (size_t)KB_QC * NP1 * 16) *
                                          sizeof(L) + 15) / 16 * 16);
  int64_t* oXq = oXlu + lup;                         // [qmax]
  int64_t* oYdr = oXq + qmax;                        // [16]
  int64_t* oYgs = oYdr + 16;                         // [16]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (nblocks + gridDim.x - 1) / gridDim.x;
  const int bend = min(nblocks, (blockIdx.x + 1) * per);
  // X fragments of one chunk for this wave's q values (ql = wave + 4i), one
  // 4-wide k step each: the next chunk's are loaded while the current one
  // is computed (at a block's last chunk, the next block's first chunk when
  // it belongs to the same descriptor).
  T xn[QPW][KS1];
  int64_t olu[KS1];   // offsets of this lane's k values in X
  int krow[KS1];      // this lane's K row (times the row pitch) per k step
  int cur = -1, pf_blk = -1;
  int64_t pf_oxr = 0;   // row offset in X of the prefetched block
  auto row_off = [&](const KbDesc& d, int blk, bool second) -> int64_t {
    const int ridx = (blk - d.tile_base) * 16 + (lane & 15);
    return ridx < d.r.size ? kb_off(d.r, ridx, second) : -1;
  };
  auto load_chunk = [&](const KbDesc& d, int64_t oxr, int q0) {
    const T* __restrict__ X = (const T*)d.X;
    const bool rok = oxr >= 0;
    const int qc = min(KB_QC, d.q.size - q0), LU = d.lu.size;
#pragma unroll
    for (int i = 0; i < QPW; ++i) {
      const int ql = wave + 4 * i;
      const int64_t oq = oXq[min(q0 + ql, qmax - 1)];
#pragma unroll
      for (int ks = 0; ks < KS1; ++ks) {
        const int k = 4 * ks + (lane >> 4);
        xn[i][ks] = (ql < qc && rok && k < LU) ? X[oxr + oq + olu[ks]] : T(0);
      }
    }
  };
  for (int blk = blockIdx.x * per; blk < bend; ++blk) {
    int lo = cur;
    if (cur < 0 || (cur + 1 < nd && ds[cur + 1].tile_base <= blk)) {
      int a = cur < 0 ? 0 : cur + 1, b = nd - 1;
      while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (ds[mid].tile_base <= blk) a = mid; else b = mid - 1;
      }
      lo = a;
    }
    const KbDesc& d = ds[lo];
    const int LU = d.lu.size, Q = d.q.size, PP = d.p.size, DR = d.dr.size, GS = d.gs.size;
    if (lo != cur) {
      __syncthreads();   // the previous descriptor's tables are no longer read
      const T* __restrict__ K = (const T*)d.K;
      const T* __restrict__ B = (const T*)d.B;
      for (int i = tid; i < lup * NP1; i += 256) {
        const int k = i / NP1, n = i - k * NP1;
        T v = T(0);
        if (k < LU && n < DR * PP)
          v = K[kb_off(d.lu, k, true) + kb_off(d.dr, n / PP, false) + kb_off(d.p, n % PP, false)];
        Ks[k * NP1PAD + n] = (L)v;
      }
      for (int i = tid; i < pqp * 16; i += 256) {
        const int k = i >> 4, c = i & 15;
        T v = T(0);
        if (k < PP * Q && c < GS) v = B[kb_off(d.p, k % PP, true) + kb_off(d.q, k / PP, true) + kb_off(d.gs, c, false)];
        Bs[k * BPAD + c] = (L)v;
      }
      for (int k = tid; k < lup; k += 256) oXlu[k] = k < LU ? kb_off(d.lu, k, false) : 0;
      for (int q = tid; q < qmax; q += 256) oXq[q] = q < Q ? kb_off(d.q, q, false) : 0;
      if (tid < 16) {
        oYdr[tid] = tid < DR ? kb_off(d.dr, tid, true) : 0;
        oYgs[tid] = tid < GS ? kb_off(d.gs, tid, true) : 0;
      }
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < KS1; ++ks) {
        const int kr = min(4 * ks + (lane >> 4), lup - 1);   // K rows clamped to the staged ones
        olu[ks] = oXlu[kr];
        krow[ks] = kr * NP1PAD + (lane & 15);
      }
      cur = lo;
      pf_blk = -1;
    }
    const int64_t oxr = pf_blk == blk ? pf_oxr : row_off(d, blk, false);
    if (pf_blk != blk) load_chunk(d, oxr, 0);
    const bool rok = oxr >= 0;
    const int64_t oyr = rok ? row_off(d, blk, true) : 0;
    typename P::Acc acc2[DRW];
#pragma unroll
    for (int t = 0; t < DRW; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc2[t][r] = 0;
    for (int q0 = 0; q0 < Q; q0 += KB_QC) {
      const int qc = min(KB_QC, Q - q0);
      T xa[QPW][KS1];
#pragma unroll
      for (int i = 0; i < QPW; ++i)
#pragma unroll
        for (int ks = 0; ks < KS1; ++ks) xa[i][ks] = xn[i][ks];
      if (q0 + KB_QC < Q) {
        load_chunk(d, oxr, q0 + KB_QC);
      } else if (blk + 1 < bend && blk + 1 - d.tile_base < (d.r.size + 15) / 16) {
        pf_oxr = row_off(d, blk + 1, false);
        load_chunk(d, pf_oxr, 0);
        pf_blk = blk + 1;
      }
      // phase 1: ket for this wave's q slots of the chunk.  Branch-free, so
      // the accumulators stay in place: slots past the chunk and k steps
      // past lu multiply zero fragments (K rows clamped to staged ones).
#pragma unroll
      for (int i = 0; i < QPW; ++i) {
        const int ql = wave + 4 * i;
        typename P::Acc acc1[NB1];
#pragma unroll
        for (int j = 0; j < NB1; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc1[j][r] = 0;
#pragma unroll
        for (int ks = 0; ks < KS1; ++ks) {
          const L* brow = Ks + krow[ks];
#pragma unroll
          for (int j = 0; j < NB1; ++j) acc1[j] = P::mma(brow[16 * j], (typename P::F)xa[i][ks], acc1[j]);
        }
        L* z = Zs + ql * NP1 * 16 + (lane & 15);
#pragma unroll
        for (int j = 0; j < NB1; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) z[(16 * j + P::row(lane, r)) * 16] = (L)acc1[j][r];
      }
      __syncthreads();
      // phase 2: bra for this wave's dr values, k = (p, q) with q fastest
      // over the chunk's KB_QC slots; p < 2, so four k steps.  The B
      // fragment and the Z row of each k step do not depend on dr: read
      // once per chunk.  Slots past the chunk, p >= PP and dr >= DR
      // contribute zeros.
      static_assert(KB_QC == 8, "q slot = k & 7");
      L bvk[4];
      int zb[4];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int k = 4 * ks + (lane >> 4);
        const int ql = k & 7, pp = k >> 3;
        const bool kok = ql < qc && pp < PP;
        zb[ks] = (kok ? ql * NP1 + pp : 0) * 16 + (lane & 15);
        bvk[ks] = kok ? Bs[(pp + PP * (q0 + ql)) * BPAD + (lane & 15)] : (L)0;
      }
#pragma unroll
      for (int t = 0; t < DRW; ++t) {
        const int dr = wave + 4 * t;
        const bool dok = dr < DR;
        const int doff = (dok ? dr : 0) * PP * 16;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) acc2[t] = P::mma(dok ? bvk[ks] : (L)0, Zs[zb[ks] + doff], acc2[t]);
      }
      __syncthreads();   // Z is rewritten by the next chunk
    }
    if (rok) {
      TC* __restrict__ Y = (TC*)d.Y;
#pragma unroll
      for (int t = 0; t < DRW; ++t) {
        const int dr = wave + 4 * t;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gs = P::row(lane, r);
          if (dr < DR && gs < GS) Y[oyr + oYdr[dr] + oYgs[gs]] = (TC)acc2[t][r];
        }
      }
    }
  }
}

int kb_lds_bytes(int prec, int nb1, int lup, int pqp, int qmax) {
  const size_t el = prec == TP_F64 ? sizeof(double) : sizeof(float);
  const size_t tiles = ((size_t)lup * kb_np1pad(nb1) + (size_t)pqp * 18 + (size_t)KB_QC * 16 * nb1 * 16) * el;
  return (int)((tiles + 15) / 16 * 16 + (size_t)(lup + qmax + 32) * sizeof(int64_t));
}

template <class P, class TC, int NB1, int KS1>
static void launch_kb_k(const KbDesc* d, int nd, int nblocks, int lup, int pqp, int qmax, int lds, hipStream_t s) {
  const int g = resident_grid(kb_kernel<P, TC, NB1, KS1>, lds, nblocks);
  kb_kernel<P, TC, NB1, KS1><<<g, 256, lds, s>>>(d, nd, nblocks, lup, pqp, qmax);
}

template <class P, class TC>
static void launch_kb_p(int nb1, const KbDesc* d, int nd, int nblocks, int lup, int pqp, int qmax, hipStream_t s) {
  const int prec = std::is_same<typename P::T, double>::value ? TP_F64 : TP_F32;
  const int lds = kb_lds_bytes(prec, nb1, lup, pqp, qmax);
  if (lup > 64) throw Error(ST_INVALID, "fused contraction: lu above 64");
  const bool short_k = lup <= 16;   // the ket's k index (lu) in at most four 4-wide steps
  if (nb1 == 1) {
    if (short_k) launch_kb_k<P, TC, 1, 4>(d, nd, nblocks, lup, pqp, qmax, lds, s);
    else launch_kb_k<P, TC, 1, 16>(d, nd, nblocks, lup, pqp, qmax, lds, s);
  } else if (nb1 == 2) {
    if (short_k) launch_kb_k<P, TC, 2, 4>(d, nd, nblocks, lup, pqp, qmax, lds, s);
    else launch_kb_k<P, TC, 2, 16>(d, nd, nblocks, lup, pqp, qmax, lds, s);
  } else {
    throw Error(ST_INVALID, "bad fused width");
  }
}

void launch_kb(int prec, int out_dt, int nb1, const KbDesc* d, int nd, int nblocks, int lup, int pqp, int qmax,
               hipStream_t s) {
  if (nblocks <= 0) return;
  if (prec == TP_F64) {
    if (out_dt != DT_F64) throw Error(ST_INVALID, "f64 contraction writes f64");
    launch_kb_p<PolF64, double>(nb1, d, nd, nblocks, lup, pqp, qmax, s);
  } else if (prec == TP_F32) {
    if (out_dt == DT_F64) launch_kb_p<PolF32, double>(nb1, d, nd, nblocks, lup, pqp, qmax, s);
    else launch_kb_p<PolF32, float>(nb1, d, nd, nblocks, lup, pqp, qmax, s);
  } else {
    throw Error(ST_INVALID, "fused contraction: f64 or f32 only");
  }
  PE_HIP(hipGetLastError());
}

// Short, skinny contraction (see TskDesc): workgroup (row tile, slice)
// stages its A block (32 x 64) and B block (64 x 32) in LDS with loads along
// each operand's unit-stride index, and wave w forms the 16 x 16 output
// block (w / 2, w % 2) on MFMA.  The slice's partial tile goes to the
// workspace through device-scope stores; the last slice of the tile to
// arrive sums all of them in slice order (its loads issued eight slices at
// a time, before the adds) and stores C.
__global__ __launch_bounds__(256) void tsk_kernel(const TskDesc* __restrict__ ds, int nd, unsigned* __restrict__ counters) {
  constexpr int MT = TSK_MT, KS = TSK_KS, AP = KS + 1, BP = 32 + 1, TE = MT * 32;
  __shared__ double As[MT * AP];
  __shared__ double Bs[KS * BP];
  __shared__ int sh;
  const int b = blockIdx.x;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ds[mid].tile_base <= b) lo = mid; else hi = mid - 1;
  }
  const TskDesc& d = ds[lo];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, lr = lane & 15, lk = lane >> 4;
  const int local = b - d.tile_base, t = local / d.ksplit, slice = local - t * d.ksplit;
  const int m0 = t * MT, k0 = slice * KS;
  const int M = d.M, N = d.N, K = d.K;
  // A block [i][kk] and B block [kk][n]: consecutive threads along each
  // operand's unit-stride index
  const bool a_kfast = d.sAk == 1 || d.sAm != 1;
  const bool b_nfast = d.sBn == 1 && d.sBk != 1;
#pragma unroll
  for (int j = 0; j < MT * KS / 256; ++j) {
    const int e = tid + 256 * j;
    const int i = a_kfast ? e / KS : e % MT, kk = a_kfast ? e % KS : e / MT;
    const int m = m0 + i, k = k0 + kk;
    As[i * AP + kk] = (m < M && k < K) ? d.A[m * d.sAm + k * d.sAk] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < KS * 32 / 256; ++j) {
    const int e = tid + 256 * j;
    const int kk = b_nfast ? e / 32 : e % KS, n = b_nfast ? e % 32 : e / KS;
    const int k = k0 + kk;
    Bs[kk * BP + n] = (n < N && k < K) ? d.B[k * d.sBk + n * d.sBn] : 0.0;
  }
  __syncthreads();
  const int bi = w >> 1, bj = w & 1;
  d4_t c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < KS / 4; ++ks)   // D = B^T A^T: lanes along the rows
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(Bs[(4 * ks + lk) * BP + 16 * bj + lr],
                                             As[(16 * bi + lr) * AP + 4 * ks + lk], c, 0, 0, 0);
  // this lane's outputs: row 16 bi + lr, columns 16 bj + lk + 4r; partial tile n-major, m fastest
  const int row = 16 * bi + lr;
  double* part = d.part + ((int64_t)t * d.ksplit + slice) * TE;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    __hip_atomic_store(&part[(16 * bj + lk + 4 * r) * MT + row], c[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __builtin_amdgcn_s_waitcnt(0);   // this thread's partial is complete before the tile's counter moves
  __syncthreads();
  if (tid == 0)
    sh = __hip_atomic_fetch_add(counters + d.cnt_base + t, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
         (unsigned)(d.ksplit - 1);
  __syncthreads();
  if (!sh) return;
  // last slice of the tile: thread -> elements tid + 256 j of the tile
  const double* tp = d.part + (int64_t)t * d.ksplit * TE;
  constexpr int PER = TE / 256;
  double acc[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) acc[j] = 0.0;
  for (int q0 = 0; q0 < d.ksplit; q0 += 8) {
    double v[8][PER];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int j = 0; j < PER; ++j)
        v[u][j] = q0 + u < d.ksplit ? __hip_atomic_load(const_cast<double*>(&tp[(int64_t)(q0 + u) * TE + tid + 256 * j]),
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                    : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)   // in slice order (a missing slice adds zero)
#pragma unroll
      for (int j = 0; j < PER; ++j) acc[j] += v[u][j];
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int e = tid + 256 * j, rr = e % MT, n = e / MT, mm = m0 + rr;
    if (mm < M && n < N) d.C[mm * d.sCm + n * d.sCn] = d.alpha * acc[j];
  }
}

void launch_tsk(const TskDesc* d, int nd, int nblocks, unsigned* counters, hipStream_t s) {
  if (nblocks <= 0) return;
  tsk_kernel<<<nblocks, 256, 0, s>>>(d, nd, counters);
  PE_HIP(hipGetLastError());
}

// Split-K reduction: one thread per output element (256 per workgroup,
// MT*NT/256 workgroups per tile); the partial slices are summed in slice
// order, so the result does not depend on scheduling.
template <class TC>
__global__ __launch_bounds__(256) void tc_reduce_kernel(const TcDesc* __restrict__ ds, int nd, int mt, int nt) {
  const int per_tile = mt * nt / 256;
  const int tile = blockIdx.x / per_tile;
  const int e = (blockIdx.x - tile * per_tile) * 256 + threadIdx.x;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ds[mid].tile_base / ds[mid].ksplit <= tile) lo = mid; else hi = mid - 1;
  }
  const TcDesc& d = ds[lo];
  const int t = tile - d.tile_base / d.ksplit;
  const int ml = e % mt, nl = e / mt;
  int m = (t / d.tiles_n) * mt + ml, n = (t % d.tiles_n) * nt + nl;
  if (m >= d.M || n >= d.N) return;
  int64_t off = 0;
  for (int j = d.nm - 1; j >= 0; --j) {
    const int dj = d.dm[j];
    off += (int64_t)(m % dj) * d.sCm[j];
    m /= dj;
  }
  for (int j = d.nn - 1; j >= 0; --j) {
    const int dj = d.dn[j];
    off += (int64_t)(n % dj) * d.sCn[j];
    n /= dj;
  }
  const int64_t sz = (int64_t)mt * nt;
  const double* __restrict__ tp = d.part + (int64_t)t * d.ksplit * sz + e;
  const int ks = d.ksplit;
  double sum = 0.0;
  int q = 0;
  for (; q + 4 <= ks; q += 4) {   // four independent loads in flight, summed in order
    const double v0 = tp[(q + 0) * sz], v1 = tp[(q + 1) * sz], v2 = tp[(q + 2) * sz], v3 = tp[(q + 3) * sz];
    sum += v0;
    sum += v1;
    sum += v2;
    sum += v3;
  }
  for (; q < ks; ++q) sum += tp[q * sz];
  TC* __restrict__ C = (TC*)d.C;
  double v = d.alpha * sum;
  if (d.beta != 0.0) v += d.beta * (double)C[off];
  C[off] = (TC)v;
}

void launch_tc_reduce(int out_dt, int tile, const TcDesc* d, int nd, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return;
  const int mt = tile_mt(tile), nt = tile_nt(tile);
  if ((mt * nt) % 256 != 0) throw Error(ST_INVALID, "bad tile");
  const int64_t grid = (int64_t)n_tiles * (mt * nt / 256);
  if (grid > INT_MAX) throw Error(ST_INVALID, "split-K reduction too large");
  if (out_dt == DT_F64) tc_reduce_kernel<double><<<(int)grid, 256, 0, s>>>(d, nd, mt, nt);
  else tc_reduce_kernel<float><<<(int)grid, 256, 0, s>>>(d, nd, mt, nt);
  PE_HIP(hipGetLastError());
}

// ===========================================================================
// Householder QR (one workgroup of 256 threads per matrix).
// ===========================================================================
constexpr int QR_MAXN = 1024;

__global__ __launch_bounds__(256) void qr_kernel(const QrDesc* __restrict__ ds) {
  const QrDesc& d = ds[blockIdx.x];
  const int m = d.m, n = d.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* __restrict__ W = d.W;                     // m x n column-major: v's and R
  double* __restrict__ V = d.W + (int64_t)m * n;    // m x n column-major: Q
  __shared__ double taus[QR_MAXN], rdiag[QR_MAXN], red[4];
  const int64_t mn = (int64_t)m * n;

  for (int64_t idx = tid; idx < mn; idx += 256) {
    const int j = (int)(idx / m), i = (int)(idx % m);
    W[idx] = d.A[i * d.sAr + j * d.sAc];
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double* wj = W + (int64_t)j * m;
    double s = 0.0;
    for (int i = j + tid; i < m; i += 256) s += wj[i] * wj[i];
    s = block_sum256(s, red);
    const double x0 = wj[j];
    const double nrm = sqrt(s);
    double beta = 0.0, tau = 0.0, scal = 0.0;
    if (nrm > 0.0) {
      beta = -copysign(nrm, x0);
      tau = (beta - x0) / beta;
      scal = 1.0 / (x0 - beta);
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < m; i += 256) wj[i] *= scal;
    if (tid == 0) { taus[j] = tau; rdiag[j] = beta; }
    __syncthreads();
    for (int k = j + 1 + wave; k < n; k += 4) {
      double* wk = W + (int64_t)k * m;
      double w = 0.0;
      for (int i = j + lane; i < m; i += 64) w += (i == j ? 1.0 : wj[i]) * wk[i];
      w = wave_sum(w) * tau;
      for (int i = j + lane; i < m; i += 64) wk[i] -= (i == j ? 1.0 : wj[i]) * w;
    }
    __syncthreads();
  }
  for (int64_t idx = tid; idx < mn; idx += 256) {
    const int j = (int)(idx / m), i = (int)(idx % m);
    V[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = n - 1; j >= 0; --j) {
    const double* wj = W + (int64_t)j * m;
    const double tau = taus[j];
    for (int k = j + wave; k < n; k += 4) {
      double* vk = V + (int64_t)k * m;
      double w = 0.0;
      for (int i = j + lane; i < m; i += 64) w += (i == j ? 1.0 : wj[i]) * vk[i];
      w = wave_sum(w) * tau;
      for (int i = j + lane; i < m; i += 64) vk[i] -= (i == j ? 1.0 : wj[i]) * w;
    }
    __syncthreads();
  }
  for (int64_t idx = tid; idx < mn; idx += 256) {
    const int j = (int)(idx / m), i = (int)(idx % m);
    const double sg = rdiag[j] < 0.0 ? -1.0 : 1.0;
    d.Q[i * d.sQr + j * d.sQc] = sg * V[idx];
  }
  if (d.R) {
    for (int idx = tid; idx < n * n; idx += 256) {
      const int j = idx / n, i = idx % n;
      const double sg = rdiag[i] < 0.0 ? -1.0 : 1.0;
      const double v = i < j ? W[(int64_t)j * m + i] : (i == j ? rdiag[i] : 0.0);
      d.R[i * d.sRr + j * d.sRc] = sg * v;
    }
  }
}

void launch_qr(const QrDesc* d, int nd, hipStream_t s) {
  if (nd <= 0) return;
  qr_kernel<<<nd, 256, 0, s>>>(d);
  PE_HIP(hipGetLastError());
}

// ===========================================================================
// Register-resident Householder QR for blocks with m <= 64*RPW, n <= NW*NCW:
// column k lives in wave k%NW (slot k/NW), row i in lane i%64 (slot i/64).
// Each reflection needs one wave reduction per trailing column and one
// barrier.  The reflectors stay in the registers of their owning wave (in
// place below the diagonal) and are broadcast through shared memory, so no
// global memory is touched between the first load and the final stores.
// ===========================================================================
// Shared memory of qr_house: 2*64*RPW + 2 + 2*NW*NCW doubles.
template <int RPW, int NCW, int NW>
__host__ __device__ constexpr int qr_house_lds() { return 2 * 64 * RPW + 2 + 2 * NW * NCW; }

template <int RPW, int NCW, int NW>
__device__ __attribute__((always_inline)) inline void qr_house(const QrDesc& d, double* sm) {
  const int m = d.m, n = d.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NMAX = NW * NCW, MMAX = 64 * RPW;
  double (*vbuf)[MMAX] = (double (*)[MMAX])sm;   // [2][MMAX]
  double* scl = sm + 2 * MMAX;                   // [2]
  double* taus = scl + 2;                        // [NMAX]
  double* rdiag = taus + NMAX;                   // [NMAX]
  double a[RPW][NCW];
#pragma unroll
  for (int s = 0; s < RPW; ++s)
#pragma unroll
    for (int c = 0; c < NCW; ++c) {
      const int i = lane + 64 * s, k = wave + NW * c;
      a[s][c] = (i < m && k < n) ? d.A[i * d.sAr + k * d.sAc] : 0.0;
    }
  // Reflection loop at run time; register slots are only ever addressed by
  // compile-time indices under uniform predicates (no dynamic indexing).
  for (int j = 0; j < n; ++j) {
    const int oc = j / NW, buf = j & 1;
    if (wave == j % NW) {
      double p = 0.0, x0loc = 0.0;
#pragma unroll
      for (int c = 0; c < NCW; ++c)
        if (c == oc) {
#pragma unroll
          for (int s = 0; s < RPW; ++s) {
            const int i = lane + 64 * s;
            if (i >= j && i < m) p += a[s][c] * a[s][c];
            if (i == j) x0loc = a[s][c];
          }
        }
      p = wave_sum(p);
      const double x0 = lane_value(x0loc, j & 63);
      const double nrm = sqrt(p);
      double beta = 0.0, tau = 0.0, scal = 0.0;
      if (nrm > 0.0) {
        beta = -copysign(nrm, x0);
        tau = (beta - x0) / beta;
        scal = 1.0 / (x0 - beta);
      }
#pragma unroll
      for (int c = 0; c < NCW; ++c)
        if (c == oc) {
#pragma unroll
          for (int s = 0; s < RPW; ++s) {
            const int i = lane + 64 * s;
            const double v = i > j ? a[s][c] * scal : (i == j ? 1.0 : 0.0);
            if (i > j) a[s][c] = v;
            vbuf[buf][i] = i < m ? v : 0.0;
          }
        }
      if (lane == 0) {
        scl[buf] = tau;
        taus[j] = tau;
        rdiag[j] = beta;
      }
    }
    __syncthreads();
    const double tau = scl[buf];
    double vi[RPW];
#pragma unroll
    for (int s = 0; s < RPW; ++s) vi[s] = vbuf[buf][lane + 64 * s];
#pragma unroll
    for (int c = 0; c < NCW; ++c) {
      const int k = wave + NW * c;
      if (k > j && k < n) {
        double p = 0.0;
#pragma unroll
        for (int s = 0; s < RPW; ++s) p += vi[s] * a[s][c];
        const double w = wave_sum(p) * tau;
#pragma unroll
        for (int s = 0; s < RPW; ++s) a[s][c] -= vi[s] * w;
      }
    }
  }
  __syncthreads();
  if (d.R) {
#pragma unroll
    for (int s = 0; s < RPW; ++s)
#pragma unroll
      for (int c = 0; c < NCW; ++c) {
        const int i = lane + 64 * s, k = wave + NW * c;
        if (i < n && k < n) {
          const double sg = rdiag[i] < 0.0 ? -1.0 : 1.0;
          const double v = i < k ? a[s][c] : (i == k ? rdiag[i] : 0.0);
          d.R[i * d.sRr + k * d.sRc] = sg * v;
        }
      }
  }
  // Q = H_0 ... H_{n-1} [I; 0], accumulated from the last reflector; the
  // owner of reflector j publishes it (unit diagonal, zeros above) each step.
  double q[RPW][NCW];
#pragma unroll
  for (int s = 0; s < RPW; ++s)
#pragma unroll
    for (int c = 0; c < NCW; ++c) q[s][c] = (lane + 64 * s == wave + NW * c) ? 1.0 : 0.0;
  for (int j = n - 1; j >= 0; --j) {
    const int oc = j / NW, buf = j & 1;
    if (wave == j % NW) {
#pragma unroll
      for (int c = 0; c < NCW; ++c)
        if (c == oc) {
#pragma unroll
          for (int s = 0; s < RPW; ++s) {
            const int i = lane + 64 * s;
            vbuf[buf][i] = (i > j && i < m) ? a[s][c] : (i == j ? 1.0 : 0.0);
          }
        }
    }
    __syncthreads();
    const double tau = taus[j];
    double vi[RPW];
#pragma unroll
    for (int s = 0; s < RPW; ++s) vi[s] = vbuf[buf][lane + 64 * s];
#pragma unroll
    for (int c = 0; c < NCW; ++c) {
      const int k = wave + NW * c;
      if (k >= j && k < n) {
        double p = 0.0;
#pragma unroll
        for (int s = 0; s < RPW; ++s) p += vi[s] * q[s][c];
        const double w = wave_sum(p) * tau;
#pragma unroll
        for (int s = 0; s < RPW; ++s) q[s][c] -= vi[s] * w;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < RPW; ++s)
#pragma unroll
    for (int c = 0; c < NCW; ++c) {
      const int i = lane + 64 * s, k = wave + NW * c;
      if (i < m && k < n) d.Q[i * d.sQr + k * d.sQc] = (rdiag[k] < 0.0 ? -1.0 : 1.0) * q[s][c];
    }
}

template <int RPW, int NCW, int NW>
__global__ __launch_bounds__(64 * NW) void qr_reg_kernel(const QrDesc* __restrict__ ds) {
  __shared__ double sm[qr_house_lds<RPW, NCW, NW>()];
  qr_house<RPW, NCW, NW>(ds[blockIdx.x], sm);
}

// ===========================================================================
// CholeskyQR2 for tall blocks (m <= 512 rows, n <= 16*NB columns), spread
// over workgroups of CQ_ROWS rows each, in three launches.  Pass 1: each
// workgroup forms the Gram matrix of its rows on MFMA (one partial tile set
// per wave, summed in wave order); the last workgroup of the block to arrive
// sums the workgroups' sets in workgroup order, factors G = R1^T R1 and
// forms W1 = R1^-1 in one wave.  Pass 2: Q1 = A W1 per workgroup (kept in
// the workspace) and the same for Q1 (G2 = R2^T R2, W2, R = R2 R1).  Pass 3:
// Q = Q1 W2.  The sums run in fixed orders, so the result does not depend on
// which workgroup arrives last.  When A is not too ill-conditioned the
// second pass makes Q orthonormal to working precision and (Q, R) agree
// with the Householder factors to the conditioning of the problem.
// Otherwise the third launch factors the block by Householder in one
// workgroup: the fallback is taken when a pivot of the first Cholesky is not
// clearly positive relative to its diagonal entry, or when an entry of
// Q1^T Q1 - I exceeds 1e-2.  Only the third launch writes Q, so Q may alias A.
//
// Wave w of a workgroup owns its rows [4*CPW*w, 4*CPW*(w+1)) and keeps two
// register images:
//   Gram image  g[c][b] = X[4*CPW*w + 4c + (lane>>4)][16b + (lane&15)]
//               (operand with k over rows: X^T X),
//   row image   x[t][s] = X[4*CPW*w + 16t + (lane&15)][4s + (lane>>4)]
//               (operand with k over columns: X W).
// Only the image whose lanes follow the smaller stride is read from memory;
// the other comes from products with 0/1 selectors, which are exact, so both
// images hold the same bits.  A product from the row image comes out of
// the MFMA as a Gram image (or, with the operands swapped, as a row image).
// ===========================================================================
__device__ inline d4_t mfma64(double x, double y, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
}

// 1/sqrt(x): hardware estimate refined by two Newton steps.
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// Selector of 4-lane groups: 1 where lane & 15 == 4*cc + (lane >> 4).
__device__ inline double cq_sel(int cc, int lane) { return (lane & 15) == 4 * cc + (lane >> 4) ? 1.0 : 0.0; }

// Row image from the Gram image.
template <int NB, int CPW>
__device__ __attribute__((always_inline)) inline void cq_to_rows(const double (&g)[CPW][NB],
                                                                 double (&x)[CPW / 4][4 * NB], int lane) {
#pragma unroll
  for (int t = 0; t < CPW / 4; ++t)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) acc = mfma64(g[4 * t + cc][b], cq_sel(cc, lane), acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) x[t][4 * b + r] = acc[r];
    }
}

// Gram image from the row image.
template <int NB, int CPW>
__device__ __attribute__((always_inline)) inline void cq_to_gram(const double (&x)[CPW / 4][4 * NB],
                                                                 double (&g)[CPW][NB], int lane) {
#pragma unroll
  for (int t = 0; t < CPW / 4; ++t)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) acc = mfma64(x[t][4 * b + sl], cq_sel(sl, lane), acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) g[4 * t + r][b] = acc[r];
    }
}

// Both images of this wave's rows of the block: the Gram image read from
// memory (GF, lanes along columns) or the row image (lanes along rows), the
// other one derived.
template <int NB, int CPW, bool GF>
__device__ __attribute__((always_inline)) inline void cq_load(const QrDesc& d, double (&g)[CPW][NB],
                                                              double (&x)[CPW / 4][4 * NB], int wave, int lane) {
  const int m = d.m, n = d.n, row0 = 4 * CPW * wave, lr = lane & 15, lk = lane >> 4;
  if (GF) {
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int i = row0 + 4 * c + lk, k = 16 * b + lr;
        g[c][b] = (i < m && k < n) ? d.A[(int64_t)i * d.sAr + (int64_t)k * d.sAc] : 0.0;
      }
    cq_to_rows<NB, CPW>(g, x, lane);
  } else {
#pragma unroll
    for (int t = 0; t < CPW / 4; ++t)
#pragma unroll
      for (int s = 0; s < 4 * NB; ++s) {
        const int i = row0 + 16 * t + lr, k = 4 * s + lk;
        x[t][s] = (i < m && k < n) ? d.A[(int64_t)i * d.sAr + (int64_t)k * d.sAc] : 0.0;
      }
    cq_to_gram<NB, CPW>(x, g, lane);
  }
}

// Partial Gram tiles (bi <= bj) of this wave's rows, written to
// part[((wave*NT + t)*4 + r)*64 + lane].
template <int NB, int CPW>
__device__ __attribute__((always_inline)) inline void cq_gram(const double (&g)[CPW][NB], double* part, int wave,
                                                              int lane) {
  constexpr int NT = NB * (NB + 1) / 2;
  int t = 0;
#pragma unroll
  for (int bi = 0; bi < NB; ++bi)
#pragma unroll
    for (int bj = bi; bj < NB; ++bj) {
      d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int c = 0; c < CPW; ++c) acc = mfma64(g[c][bi], g[c][bj], acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) part[((wave * NT + t) * 4 + r) * 64 + lane] = acc[r];
      ++t;
    }
}

// Sum of the eight partial tile sets in wave order, stored as the full
// symmetric matrix G[i*(NP+1) + j] over the partial area (all threads).
template <int NB>
__device__ __attribute__((always_inline)) inline void cq_reduce(double* part, int tid) {
  constexpr int NT = NB * (NB + 1) / 2, NE = NT * 256, PER = (NE + 511) / 512, LD = 16 * NB + 1;
  double v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + 512 * q;
    v[q] = 0.0;
    if (e < NE)
#pragma unroll
      for (int w = 0; w < 8; ++w) v[q] += part[w * NE + e];
  }
  __syncthreads();   // every partial is read before G overwrites them
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + 512 * q;
    if (e < NE) {
      int t = e >> 8, bi = 0;
      while (t >= NB - bi) {
        t -= NB - bi;
        ++bi;
      }
      const int bj = bi + t, l = e & 63, r = (e >> 6) & 3;
      const int i = 16 * bi + (l >> 4) + 4 * r, j = 16 * bj + (l & 15);
      part[i * LD + j] = v[q];
      if (bi != bj) part[j * LD + i] = v[q];
    }
  }
  __syncthreads();
}

// 1/x: hardware estimate e0 = 1 - x*y0, corrected to third order,
// y0 (1 + e0 + e0^2), and returned as f*y0 with f supplied by the caller.
__device__ inline double rcp_scaled(double x, double f) {
  const double y0 = __builtin_amdgcn_rcp(x);
  const double e0 = fma(-x, y0, 1.0);
  const double t = f * y0;
  return fma(t, fma(e0, e0, e0), t);
}

// One wave: Cholesky G = R^T R (R upper, positive diagonal) and W = R^-1 by
// Gauss-Jordan elimination on [G | I].  Lane j < NP holds column j of G,
// lane NP + j column j of I, so each row operation is one instruction over
// the wave.  Rows are eliminated unscaled (G = L D L^T with pivots p_k): the
// multiplier for row i at step k is G[i][k]/p_k, taken as G[k][i]/p_k by the
// symmetry of the trailing block, i.e. lane i's entry of row k.  The next
// pivot's row is updated at once (that multiplier by readlane), the other
// rows one step later with multipliers published through row[0..128) (two
// buffers).  At
// the end row k of both halves is scaled by p_k^-1/2 (one inverse square
// root per lane), which turns D^-1/2 U into R and L^-T D^-1/2 into W.
// Columns j >= nv are unit columns.  Returns false when a pivot is not above
// tol times its original diagonal entry (or not finite), or, for devmax > 0,
// when an entry of G - I exceeds devmax.  Writes R[k*(NP+1) + j] and
// W[j*(NP+1) + k], zeros below the diagonal; uses row[0..128 + NP).
template <int NB>
__device__ __attribute__((always_inline)) inline bool cq_chol(const double* G, double* R, double* W, double* row,
                                                              int nv, double tol, double devmax, int lane) {
  constexpr int NP = 16 * NB, LD = NP + 1;
  const bool gp = lane < NP, act = lane < 2 * NP;
  const int j = gp ? lane : (act ? lane - NP : 0);
  const bool real = gp && j < nv;
  double* piv = row + 128;
  double g[NP];
  bool bad = false;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const double gv = G[i * LD + j];   // a valid address on every lane: no branch per load
    const double unit = (act && i == j) ? 1.0 : 0.0;
    g[i] = real ? (i < nv ? gv : 0.0) : unit;
    if (devmax > 0.0 && real && i < nv && !(fabs(gv - unit) <= devmax)) bad = true;
  }
  double mp[NP];        // lane i's entry of the previous row, for its deferred updates
  double sprev = 0.0;   // the previous row divided by its pivot (this lane's entry)
#pragma unroll
  for (int i = 0; i < NP; ++i) mp[i] = 0.0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const double p = lane_value(g[k], k);
    const double gk = g[k];
    const double sk = rcp_scaled(p, gk);   // row k / p_k
    double* rb = row + 64 * (k & 1);
    rb[lane] = gk;
    piv[k] = p;                            // the same value from every lane
    if (k + 1 < NP) g[k + 1] = fma(-lane_value(gk, k + 1), sk, g[k + 1]);
#pragma unroll
    for (int i = k + 1; i < NP; ++i)
      if (k >= 1) g[i] = fma(-mp[i], sprev, g[i]);   // row k-1, rows after the pivot's
#pragma unroll
    for (int i = k + 2; i < NP; ++i) mp[i] = rb[i];
    __builtin_amdgcn_sched_barrier(1);   // keep these reads here (ALU work may still move across)
    sprev = sk;
  }
  // pivot checks and p_k^-1/2 (lane k), published in row[0..NP)
  if (gp) {
    const double p = piv[lane];
    if (real && !(p > tol * G[j * LD + j] && p <= 1.0e300)) bad = true;
    row[lane] = rsqrt_nr(p);
  }
  if (act) {
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const bool keep = gp ? k <= j : j <= k;
      (gp ? R[k * LD + j] : W[j * LD + k]) = keep ? g[k] * row[k] : 0.0;
    }
  }
  return !__any(bad);
}

// Gram image of X W (W upper triangular, W[k*(NP+1) + c] in shared memory).
template <int NB, int CPW>
__device__ __attribute__((always_inline)) inline void cq_right(const double (&x)[CPW / 4][4 * NB], const double* W,
                                                               double (&g)[CPW][NB], int lane) {
  constexpr int LD = 16 * NB + 1;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int bj = 0; bj < NB; ++bj) {
    double wf[4 * NB];
#pragma unroll
    for (int s = 0; s < 4 * (bj + 1); ++s) wf[s] = W[(4 * s + lk) * LD + 16 * bj + lr];
#pragma unroll
    for (int t = 0; t < CPW / 4; ++t) {
      d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4 * (bj + 1); ++s) acc = mfma64(x[t][s], wf[s], acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) g[4 * t + r][bj] = acc[r];
    }
  }
}

// Q = X W stored to d.Q: from the Gram image of the product (BC, lanes
// along columns of Q) or from its row image (operands swapped, lanes along
// rows).
template <int NB, int CPW, bool BC>
__device__ __attribute__((always_inline)) inline void cq_store_q(const QrDesc& d, const double (&x)[CPW / 4][4 * NB],
                                                                 const double* W, int wave, int lane) {
  constexpr int LD = 16 * NB + 1;
  const int m = d.m, n = d.n, row0 = 4 * CPW * wave, lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int bj = 0; bj < NB; ++bj) {
    double wf[4 * NB];
#pragma unroll
    for (int s = 0; s < 4 * (bj + 1); ++s) wf[s] = W[(4 * s + lk) * LD + 16 * bj + lr];
#pragma unroll
    for (int t = 0; t < CPW / 4; ++t) {
      d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4 * (bj + 1); ++s) acc = BC ? mfma64(x[t][s], wf[s], acc) : mfma64(wf[s], x[t][s], acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = row0 + 16 * t + (BC ? lk + 4 * r : lr), k = 16 * bj + (BC ? lr : lk + 4 * r);
        if (i < m && k < n) d.Q[(int64_t)i * d.sQr + (int64_t)k * d.sQc] = acc[r];
      }
    }
  }
}

// R = R2 R1 on MFMA: wave w < NB*NB forms the 16x16 tile (w / NB, w % NB);
// entries below the diagonal are stored as zeros.
template <int NB>
__device__ __attribute__((always_inline)) inline void cq_store_r(const QrDesc& d, const double* R2, const double* R1,
                                                                 int wave, int lane) {
  constexpr int LD = 16 * NB + 1;
  if (wave >= NB * NB) return;
  const int n = d.n, bi = wave / NB, bj = wave - bi * NB, lr = lane & 15, lk = lane >> 4;
  d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < 4 * NB; ++s)
    acc = mfma64(R2[(16 * bi + lr) * LD + 4 * s + lk], R1[(4 * s + lk) * LD + 16 * bj + lr], acc);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = 16 * bi + lk + 4 * r, j = 16 * bj + lr;
    if (i < n && j < n) d.R[(int64_t)i * d.sRr + (int64_t)j * d.sRc] = i <= j ? acc[r] : 0.0;
  }
}

// Workspace of one block (doubles): the workgroups' partial Gram tile sets
// of pass 1, then those of pass 2.
size_t cq_ws_doubles(int m, int n) {
  const int NB = n <= 16 ? 1 : 2, P = (m + CQ_ROWS - 1) / CQ_ROWS;
  return (size_t)2 * P * (NB * (NB + 1) / 2) * 256;
}

// The block whose workgroup range holds workgroup b, and b's index in it.
__device__ inline const CqDesc& cq_find(const CqDesc* ds, int nd, int b, int& p) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ds[mid].block_base <= b) lo = mid; else hi = mid - 1;
  }
  p = b - ds[lo].block_base;
  return ds[lo];
}

// This workgroup's rows of a block as a block of their own.
__device__ inline QrDesc cq_rows(const QrDesc& d, int p) {
  QrDesc q = d;
  q.A = d.A + (int64_t)CQ_ROWS * p * d.sAr;
  q.Q = d.Q + (int64_t)CQ_ROWS * p * d.sQr;
  q.m = min(CQ_ROWS, d.m - CQ_ROWS * p);
  return q;
}

// Data that workgroups of one block exchange (their partial Gram sets) is
// written and read with device-scope accesses, which bypass the
// per-XCD L2 caches' stale copies, so no cache-wide write-back or
// invalidation is needed: a writer waits for its stores to complete before
// the counter moves, and a reader loads after it has seen the counter move.
__device__ inline void cq_st(double* p, double v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline double cq_ld(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Arrival at the block's counter: the value before this workgroup's
// increment (its device-scope stores before the call are complete).
__device__ inline unsigned cq_arrive(unsigned* c, int* sh) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) *sh = (int)__hip_atomic_fetch_add(c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const unsigned old = (unsigned)*sh;
  __syncthreads();
  return old;
}

// Wait until the counter reaches `target` (every workgroup of the block has
// stored its partial Gram set).  Every workgroup of a launch is resident (at
// most CQ_MAXWG of them, one per compute unit), so the wait ends; the polls
// are bounded all the same, and a wait that runs out returns false.
__device__ inline bool cq_wait(unsigned* c, unsigned target, int* sh) {
  if (threadIdx.x == 0) {
    int ok = 0;
    for (int it = 0; it < (1 << 20); ++it) {
      if (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) {
        ok = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    *sh = ok;
  }
  __syncthreads();
  const bool ok = *sh != 0;
  __syncthreads();
  return ok;
}

// A wait that ran out: this workgroup's rows of Q become NaN, which the
// callers' finiteness checks report.
__device__ inline void cq_poison(const QrDesc& q) {
  for (int e = threadIdx.x; e < q.m * q.n; e += blockDim.x)
    q.Q[(int64_t)(e / q.n) * q.sQr + (int64_t)(e % q.n) * q.sQc] = __builtin_nan("");
}

// Partial Gram tile set of one workgroup (the eight waves' sets in sm,
// summed in wave order) to its slot of the workspace.
template <int NB>
__device__ inline void cq_put_part(const double* sm, double* part, int p, int tid) {
  constexpr int NE = NB * (NB + 1) / 2 * 256;
  for (int e = tid; e < NE; e += 512) {
    double v = sm[e];
#pragma unroll
    for (int w = 1; w < 8; ++w) v += sm[w * NE + e];
    cq_st(&part[(int64_t)p * NE + e], v);
  }
}

// Sum of the P <= CQ_MAXP workgroups' tile sets in workgroup order, stored
// as the full symmetric matrix G[i*(NP+1) + j] (512 threads; all loads are
// issued before the first add).
template <int NB>
__device__ inline void cq_sum_parts(const double* part, int P, double* G, int tid) {
  constexpr int NT = NB * (NB + 1) / 2, NE = NT * 256, LD = 16 * NB + 1, PER = (NE + 511) / 512;
  double v[PER][CQ_MAXP];
#pragma unroll
  for (int q = 0; q < PER; ++q)
#pragma unroll
    for (int w = 0; w < CQ_MAXP; ++w) {
      const int e = tid + 512 * q;
      v[q][w] = (w < P && e < NE) ? cq_ld(&part[(int64_t)w * NE + e]) : 0.0;
    }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + 512 * q;
    if (e >= NE) continue;
    double s = v[q][0];
#pragma unroll
    for (int w = 1; w < CQ_MAXP; ++w) s += v[q][w];   // zeros past P leave the sum unchanged
    int t = e >> 8, bi = 0;
    while (t >= NB - bi) {
      t -= NB - bi;
      ++bi;
    }
    const int bj = bi + t, l = e & 63, r = (e >> 6) & 3;
    const int i = 16 * bi + (l >> 4) + 4 * r, j = 16 * bj + (l & 15);
    G[i * LD + j] = s;
    if (bi != bj) G[j * LD + i] = s;
  }
}

constexpr int CQ_CPW = CQ_ROWS / 32;   // row chunks of 4 per wave (eight waves)
static_assert(CQ_CPW % 4 == 0, "whole 16-row tiles per wave");

// One launch per group of blocks, all workgroups resident.  A block's
// counter (zero at launch) counts the P arrivals after pass 1 and the P
// after pass 2.  Every workgroup waits for all P arrivals of a pass, sums
// the P partial Gram sets itself in workgroup order and runs the same
// Cholesky, so all of them hold the same factors (bit for bit) without any
// factor being published.  After a failed check (the same in every
// workgroup) the first workgroup factors the whole block by Householder
// (A is untouched until pass 3) and the others leave.
template <int NB>
__global__ __launch_bounds__(512) void cq_kernel(const CqDesc* __restrict__ ds, int nd, unsigned* __restrict__ counters) {
  constexpr int CPW = CQ_CPW, NP = 16 * NB, LD = NP + 1, NT = NB * (NB + 1) / 2;
  // LDS: G, R, W and the row buffers of the Cholesky overlap the waves'
  // partial tile sets (consumed before each sum); R1 lies past both
  constexpr int A1 = NP * LD + 8 * NT * 256, A2 = 3 * NP * LD + 128 + NP, A3 = qr_house_lds<8, 2 * NB, 8>();
  constexpr int A12 = A1 > A2 ? A1 : A2;
  constexpr int AREA = (A12 + NP * LD) > A3 ? A12 + NP * LD : A3;
  __shared__ double sm[AREA];
  __shared__ int sh;
  int p;
  const CqDesc& d = cq_find(ds, nd, blockIdx.x, p);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int P = d.P;
  unsigned* cnt = counters + d.cnt;
  double* part = d.ws;
  double *Gs = sm, *Rs = sm + NP * LD, *Ws = sm + 2 * NP * LD, *rowb = sm + 3 * NP * LD;
  double* R1s = sm + A12;          // R1, kept for R = R2 R1
  double* wpart = sm + NP * LD;    // the waves' partial tile sets (before the sum)
  const QrDesc q = cq_rows(d.q, p);
  double g[CPW][NB], x[CPW / 4][4 * NB];
  if ((d.q.sAc < 0 ? -d.q.sAc : d.q.sAc) <= (d.q.sAr < 0 ? -d.q.sAr : d.q.sAr))
    cq_load<NB, CPW, true>(q, g, x, wave, lane);
  else
    cq_load<NB, CPW, false>(q, g, x, wave, lane);
  // ---- pass 1: G = A^T A, R1, W1 (in Ws)
  cq_gram<NB, CPW>(g, wpart, wave, lane);
  __syncthreads();
  cq_put_part<NB>(wpart, part, p, tid);
  cq_arrive(cnt, &sh);
  if (!cq_wait(cnt, (unsigned)P, &sh)) {
    cq_poison(q);
    return;
  }
  cq_sum_parts<NB>(part, P, Gs, tid);
  __syncthreads();
  if (wave == 0) {
    const bool good = cq_chol<NB>(Gs, Rs, Ws, rowb, d.q.n, 1e-14, 0.0, lane);
    if (lane == 0) sh = good;
  }
  __syncthreads();
  if (!sh) {
    if (p == 0) qr_house<8, 2 * NB, 8>(d.q, sm);
    return;
  }
  for (int e = tid; e < NP * LD; e += 512) R1s[e] = Rs[e];
  // ---- pass 2: Q1 = A W1 (kept in registers), G2 = Q1^T Q1, W2, R = R2 R1
  cq_right<NB, CPW>(x, Ws, g, lane);
  __syncthreads();   // W1 and R1 are read before the partial tiles reuse the area
  cq_gram<NB, CPW>(g, wpart, wave, lane);
  __syncthreads();
  // this pass's partial sets go to the second half of the block's area
  cq_put_part<NB>(wpart, part + (int64_t)P * NT * 256, p, tid);
  cq_arrive(cnt, &sh);
  if (!cq_wait(cnt, 2 * (unsigned)P, &sh)) {
    cq_poison(q);
    return;
  }
  cq_sum_parts<NB>(part + (int64_t)P * NT * 256, P, Gs, tid);
  __syncthreads();
  if (wave == 0) {
    const bool good = cq_chol<NB>(Gs, Rs, Ws, rowb, d.q.n, 0.5, 1e-2, lane);
    if (lane == 0) sh = good;
  }
  __syncthreads();
  if (!sh) {
    if (p == 0) qr_house<8, 2 * NB, 8>(d.q, sm);
    return;
  }
  if (p == 0 && d.q.R) cq_store_r<NB>(d.q, Rs, R1s, wave, lane);
  // ---- pass 3: Q = Q1 W2
  cq_to_rows<NB, CPW>(g, x, lane);
  if ((d.q.sQc < 0 ? -d.q.sQc : d.q.sQc) <= (d.q.sQr < 0 ? -d.q.sQr : d.q.sQr))
    cq_store_q<NB, CPW, true>(q, x, Ws, wave, lane);
  else
    cq_store_q<NB, CPW, false>(q, x, Ws, wave, lane);
}

__global__ void cq_clear_kernel(unsigned* c, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = 0u;
}

void launch_cq_clear(unsigned* counters, int n, hipStream_t s) {
  if (n <= 0) return;
  cq_clear_kernel<<<(n + 255) / 256, 256, 0, s>>>(counters, n);
  PE_HIP(hipGetLastError());
}

void launch_cq(int nb, const CqDesc* d, int nd, int nblocks, unsigned* counters, hipStream_t s) {
  PE_REQUIRE(nb == 1 || nb == 2, "CholeskyQR2: bad column-block count");
  PE_REQUIRE(nblocks <= CQ_MAXWG, "CholeskyQR2: too many workgroups in one launch");
  if (nb == 1) cq_kernel<1><<<nblocks, 512, 0, s>>>(d, nd, counters);
  else cq_kernel<2><<<nblocks, 512, 0, s>>>(d, nd, counters);
  PE_HIP(hipGetLastError());
}

// Register-resident variants: (rows per lane, columns per wave, waves).
// Sixteen waves keep two or fewer columns per wave for n <= 32, which
// shortens the per-reflection critical path.  A lane holds its block
// entries and the same number of Q entries: at 16 waves per workgroup
// (128 VGPRs per lane) that allows 16 entries each, at 8 waves 32.
struct QrVariant {
  int rpw, ncw, nw;
};
constexpr QrVariant QR_VARIANTS[] = {{1, 2, 4},  {1, 4, 4},  {1, 1, 16}, {2, 1, 16}, {4, 1, 16},
                                     {8, 1, 16}, {16, 2, 8}, {2, 2, 16}, {4, 2, 16},
                                     {8, 2, 16}, {4, 4, 16}, {4, 5, 16}};
constexpr int QR_NVAR = sizeof(QR_VARIANTS) / sizeof(QR_VARIANTS[0]);

int qr_variant_for(int m, int n) {
  if (m >= 128 && m >= 4 * n && m <= 512 && n <= 32) return QR_CQ;
  int best = -1, cost = 1 << 30;
  for (int v = 0; v < QR_NVAR; ++v) {
    const QrVariant& q = QR_VARIANTS[v];
    const int c = q.rpw * q.ncw * 4 + (q.nw == 16 ? 1 : 0);   // registers, then fewer waves
    if (64 * q.rpw >= m && q.nw * q.ncw >= n && c < cost) {
      best = v;
      cost = c;
    }
  }
  return best;   // -1: use the streaming kernel
}

void launch_qr_reg(int variant, const QrDesc* d, int nd, hipStream_t s) {
  switch (variant) {
    case 0: qr_reg_kernel<1, 2, 4><<<nd, 256, 0, s>>>(d); break;
    case 1: qr_reg_kernel<1, 4, 4><<<nd, 256, 0, s>>>(d); break;
    case 2: qr_reg_kernel<1, 1, 16><<<nd, 1024, 0, s>>>(d); break;
    case 3: qr_reg_kernel<2, 1, 16><<<nd, 1024, 0, s>>>(d); break;
    case 4: qr_reg_kernel<4, 1, 16><<<nd, 1024, 0, s>>>(d); break;
    case 5: qr_reg_kernel<8, 1, 16><<<nd, 1024, 0, s>>>(d); break;
    case 6: qr_reg_kernel<16, 2, 8><<<nd, 512, 0, s>>>(d); break;
    case 7: qr_reg_kernel<2, 2, 16><<<nd, 1024, 0, s>>>(d); break;
    case 8: qr_reg_kernel<4, 2, 16><<<nd, 1024, 0, s>>>(d); break;
    case 9: qr_reg_kernel<8, 2, 16><<<nd, 1024, 0, s>>>(d); break;
    case 10: qr_reg_kernel<4, 4, 16><<<nd, 1024, 0, s>>>(d); break;
    case 11: qr_reg_kernel<4, 5, 16><<<nd, 1024, 0, s>>>(d); break;
    default: throw Error(ST_INVALID, "bad QR variant");
  }
  PE_HIP(hipGetLastError());
}

// ===========================================================================
// Two-pass deterministic reductions.
// ===========================================================================
template <class T>
__device__ inline double ldv(const void* p, int64_t i) { return (double)((const T*)p)[i]; }

__global__ __launch_bounds__(256) void red1_kernel(const RedDesc* __restrict__ ds, int nd, double* partials) {
  __shared__ double red[4];
  const int bid = blockIdx.x;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ds[mid].block_base <= bid) lo = mid; else hi = mid - 1;
  }
  const RedDesc& d = ds[lo];
  const int b = bid - d.block_base;
  const int64_t chunk = (d.n + d.nblocks - 1) / d.nblocks;
  const int64_t i0 = b * chunk, i1 = min(d.n, i0 + chunk);
  double s = 0.0;
  if (d.dt == DT_F64) {
    if (d.y) for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) s += ldv<double>(d.x, i) * ldv<double>(d.y, i);
    else for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) { const double v = ldv<double>(d.x, i); s += v * v; }
  } else {
    if (d.y) for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) s += ldv<float>(d.x, i) * ldv<float>(d.y, i);
    else for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) { const double v = ldv<float>(d.x, i); s += v * v; }
  }
  s = block_sum256(s, red);
  if (threadIdx.x == 0) partials[d.part_base + b] = s;
}

__global__ void red2_kernel(const RedDesc* __restrict__ ds, const double* __restrict__ partials) {
  const RedDesc& d = ds[blockIdx.x];
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < d.nblocks; ++b) s += partials[d.part_base + b];
    *d.out = s;
  }
}

void launch_reduce(const RedDesc* d, int nd, int nb, double* partials, hipStream_t s) {
  if (nd <= 0) return;
  red1_kernel<<<nb, 256, 0, s>>>(d, nd, partials);
  red2_kernel<<<nd, 64, 0, s>>>(d, partials);
  PE_HIP(hipGetLastError());
}

// ===========================================================================
// Elementwise kernels.
// ===========================================================================
__device__ inline double ew_load(const void* p, int dt, int64_t i) {
  return dt == DT_F64 ? ((const double*)p)[i] : (double)((const float*)p)[i];
}
__device__ inline void ew_store(void* p, int dt, int64_t i, double v) {
  if (dt == DT_F64) ((double*)p)[i] = v; else ((float*)p)[i] = (float)v;
}

__global__ __launch_bounds__(256) void ew_kernel(const EwDesc* __restrict__ ds, int nd) {
  const int bid = blockIdx.x;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ds[mid].block_base <= bid) lo = mid; else hi = mid - 1;
  }
  const EwDesc& d = ds[lo];
  const int64_t stride = (int64_t)d.nblocks * 256;
  const int64_t n = d.n;
  if (d.kind == EW_LOGACC) {   // a short sequential sum (one per boundary side)
    if (bid == d.block_base && threadIdx.x == 0) {
      const double* const* w = (const double* const*)d.src;
      double* out = (double*)d.dst;
      double acc = 0.0;
      out[0] = 0.0;
      for (int64_t k = 0; k < n; ++k) {
        acc += 0.5 * log(*w[k]);
        out[k + 1] = acc;
      }
    }
    return;
  }
  if (d.kind == EW_NONFINITE) {   // every writer stores the same value
    for (int64_t i = (int64_t)(bid - d.block_base) * 256 + threadIdx.x; i < n; i += stride)
      if (!isfinite(ew_load(d.src, d.src_dt, i))) ((double*)d.dst)[0] = d.a;
    return;
  }
  for (int64_t i = (int64_t)(bid - d.block_base) * 256 + threadIdx.x; i < n; i += stride) {
    double v;
    switch (d.kind) {
      case EW_COPY: v = ew_load(d.src, d.src_dt, i); break;
      case EW_PHYS: {
        const int64_t Lh = n / 2, j = i % Lh;
        const int p = (int)(i / Lh);
        v = d.op[2 * p] * ew_load(d.src, d.src_dt, j) + d.op[2 * p + 1] * ew_load(d.src, d.src_dt, Lh + j);
        break;
      }
      case EW_FILL: v = d.a; break;
      case EW_SPLITMIX: {
        const uint64_t x = splitmix_mix(d.key + (uint64_t)(i + 1) * SPLITMIX_GAMMA);
        v = (double)(x >> 11) * 0x1.0p-53 * 2.0 - 1.0;
        break;
      }
      case EW_RSQRT: v = ew_load(d.src, d.src_dt, i) / sqrt(*d.sptr); break;
      case EW_IDENTITY: v = (i / d.dim == i % d.dim) ? d.a : 0.0; break;
      default: v = 0.0;
    }
    ew_store(d.dst, d.dst_dt, i, v);
  }
}

void launch_ew(const EwDesc* d, int nd, int nb, hipStream_t s) {
  if (nd <= 0) return;
  ew_kernel<<<nb, 256, 0, s>>>(d, nd);
  PE_HIP(hipGetLastError());
}


// ===========================================================================
// CU_0 separable boundaries (one workgroup per lattice direction).
//
// Every site step contracts one site's two layers with D x D matrices on its
// four legs, O(d D^5) per step (Sec. 5.1).  The steps of a direction form
// one long dependent chain (rows, sweeps, sites), so the kernel is built for
// latency: one 1024-thread workgroup per direction; the site tensor, the
// matrices on its legs and the two intermediates live in LDS, every virtual
// leg padded with zeros to the direction's largest bond DM (a template
// argument, so index arithmetic is by constants; the zeros change no sum);
// the final contraction over four legs (DM^2 outputs by d DM^3 terms) is
// split over all threads in fixed slices, summed in slice order.  The b of a
// site and the environment update in the same direction share their first
// two contractions.
// ===========================================================================
namespace {

constexpr int SEP_V = SEP_MAXD * SEP_MAXD;            // one D x D matrix slot
constexpr int SEP_T = 1024;                           // threads per workgroup

struct SepSh {
  double* A;      // staged site [p][l][u][r][d], legs padded to DM
  double* W1;
  double* W2;
  double* part;   // SEP_T partial sums
  double* B;      // DM x DM
  double* red;    // SEP_T / 64
  double* e;      // the step's left, up, right and down matrices, DM x DM each
  double* su;
  double* f;
  double* sg;
};

__device__ inline double sepA(const SepSite& s, int p, int l, int u, int r, int d) {
  return s.A[p * s.sp + l * s.sl + u * s.su + r * s.sr + d * s.sd];
}

__device__ inline double sep_block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < SEP_T / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Copy an n x n matrix (row stride n) into a zero-padded DM x DM one.
template <int DM>
__device__ inline void sep_pad(double* dst, const double* src, int n) {
  const int i = threadIdx.x;
  if (i < DM * DM) {
    const int a = i / DM, b = i % DM;
    dst[i] = (a < n && b < n) ? src[a * n + b] : 0.0;
  }
}

// Stage one site step's operands in LDS (null matrices: not needed by this
// step; `pad_env` false: e and f are already padded DM x DM slots).
template <int DM>
__device__ void sep_stage(const SepSite& s, const SepSh& sh, const double* e, const double* su, const double* f,
                          const double* sg) {
  constexpr int V4 = DM * DM * DM * DM;
  const int n = s.d * V4;
  for (int i = threadIdx.x; i < n; i += SEP_T) {
    const int d = i % DM, r = (i / DM) % DM, u = (i / (DM * DM)) % DM, l = (i / (DM * DM * DM)) % DM, p = i / V4;
    sh.A[i] = (l < s.Dl && u < s.Du && r < s.Dr && d < s.Dd) ? sepA(s, p, l, u, r, d) : 0.0;
  }
  const int i = threadIdx.x;
  if (e && i < DM * DM) sh.e[i] = e[i];
  if (f && i < DM * DM) sh.f[i] = f[i];
  if (su) sep_pad<DM>(sh.su, su, s.Du);
  if (sg) sep_pad<DM>(sh.sg, sg, s.Dd);
  __syncthreads();
}

// out[o] = sum over q < K of term(o, q) for o < DM^2: thread t takes output
// t % DM^2 over the (t / DM^2)-th of SEP_T / DM^2 equal slices of q; the
// slices are then summed in order.
template <int DM, class F>
__device__ void sep_reduce(int K, double* part, double* out, F term) {
  constexpr int NO = DM * DM, ns = SEP_T / NO;
  const int t = threadIdx.x;
  if (t < ns * NO) {
    const int o = t % NO, j = t / NO;
    const int qa = (K * j) / ns, qb = (K * (j + 1)) / ns;
    double acc = 0.0;
    for (int q = qa; q < qb; ++q) acc += term(o, q);
    part[t] = acc;
  }
  __syncthreads();
  if (t < NO) {
    double acc = 0.0;
    for (int j = 0; j < ns; ++j) acc += part[j * NO + t];
    out[t] = acc;
  }
  __syncthreads();
}

// Scale x[0..n) to unit Frobenius norm (every thread of the block calls this).
__device__ void sep_unit(double* x, int n, double* red) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += SEP_T) s += x[i] * x[i];
  s = sep_block_sum(s, red);
  const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (int i = threadIdx.x; i < n; i += SEP_T) x[i] *= inv;
  __syncthreads();
}

// Left half of a site step: W2[p][m][v][r][d] = sum e[l][m] su[u][v] A[p,l,u,r,d]
template <int DM>
__device__ void sep_left(int P, const SepSh& sh) {
  const int n = P * DM * DM * DM * DM;
  for (int i = threadIdx.x; i < n; i += SEP_T) {   // W1[p][m][u][r][d] = sum_l e[l][m] A[p,l,u,r,d]
    const int urd = i % (DM * DM * DM), m = (i / (DM * DM * DM)) % DM, p = i / (DM * DM * DM * DM);
    double acc = 0.0;
#pragma unroll
    for (int l = 0; l < DM; ++l) acc += sh.e[l * DM + m] * sh.A[(p * DM + l) * DM * DM * DM + urd];
    sh.W1[i] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += SEP_T) {   // W2[p][m][v][r][d] = sum_u W1[p][m][u][r][d] su[u][v]
    const int rd = i % (DM * DM), v = (i / (DM * DM)) % DM, pm = i / (DM * DM * DM);
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < DM; ++u) acc += sh.W1[(pm * DM + u) * DM * DM + rd] * sh.su[u * DM + v];
    sh.W2[i] = acc;
  }
  __syncthreads();
}

// Right half: W2[p][l][v][s][d] = sum f[r][s] su[u][v] A[p,l,u,r,d]
template <int DM>
__device__ void sep_right(int P, const SepSh& sh) {
  const int n = P * DM * DM * DM * DM;
  for (int i = threadIdx.x; i < n; i += SEP_T) {   // W1[p][l][u][s][d] = sum_r A[p,l,u,r,d] f[r][s]
    const int d = i % DM, ss = (i / DM) % DM, plu = i / (DM * DM);
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < DM; ++r) acc += sh.A[(plu * DM + r) * DM + d] * sh.f[r * DM + ss];
    sh.W1[i] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += SEP_T) {   // W2[p][l][v][s][d] = sum_u W1[p][l][u][s][d] su[u][v]
    const int sd = i % (DM * DM), v = (i / (DM * DM)) % DM, pl = i / (DM * DM * DM);
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < DM; ++u) acc += sh.W1[(pl * DM + u) * DM * DM + sd] * sh.su[u * DM + v];
    sh.W2[i] = acc;
  }
  __syncthreads();
}

// b[d][g] = sum_{p,m,v,s} W1[p][m][v][s][d] A[p,m,v,s,g] (W1 made by the caller)
template <int DM>
__device__ void sep_b_final(int P, const SepSh& sh, double* out) {
  const double* W = sh.W1;
  const double* A = sh.A;
  sep_reduce<DM>(P * DM * DM * DM, sh.part, out, [&](int o, int q) {
    const int d = o / DM, g = o % DM;
    return W[q * DM + d] * A[q * DM + g];
  });
}

// b from the left half in W2: W1[p][m][v][s][d] = sum_r W2[p][m][v][r][d] f[r][s]
template <int DM>
__device__ void sep_b_from_left(int P, const SepSh& sh, double* out) {
  const int n = P * DM * DM * DM * DM;
  for (int i = threadIdx.x; i < n; i += SEP_T) {
    const int d = i % DM, ss = (i / DM) % DM, pmv = i / (DM * DM);
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < DM; ++r) acc += sh.W2[(pmv * DM + r) * DM + d] * sh.f[r * DM + ss];
    sh.W1[i] = acc;
  }
  __syncthreads();
  sep_b_final<DM>(P, sh, out);
}

// b from the right half in W2: W1[p][m][v][s][d] = sum_l e[l][m] W2[p][l][v][s][d]
template <int DM>
__device__ void sep_b_from_right(int P, const SepSh& sh, double* out) {
  constexpr int V3 = DM * DM * DM;
  const int n = P * DM * V3;
  for (int i = threadIdx.x; i < n; i += SEP_T) {
    const int vsd = i % V3, m = (i / V3) % DM, p = i / (DM * V3);
    double acc = 0.0;
#pragma unroll
    for (int l = 0; l < DM; ++l) acc += sh.e[l * DM + m] * sh.W2[(p * DM + l) * V3 + vsd];
    sh.W1[i] = acc;
  }
  __syncthreads();
  sep_b_final<DM>(P, sh, out);
}

// W1[...][g] = sum_d W2[...][d] sig[d][g] (the last leg contracted with sigma)
template <int DM>
__device__ void sep_close_down(int P, const SepSh& sh, const double* sg) {
  const int n = P * DM * DM * DM * DM;
  for (int i = threadIdx.x; i < n; i += SEP_T) {
    const int g = i % DM, base = i - g;
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < DM; ++d) acc += sh.W2[base + d] * sg[d * DM + g];
    sh.W1[i] = acc;
  }
  __syncthreads();
}

// e'[r][s] from the left half in W2 = sum_{p,m,v,g} (W2 sig)[p][m][v][r][g] A[p,m,v,s,g]
template <int DM>
__device__ void sep_e_from_left(int P, const SepSh& sh, const double* sg, double* out) {
  sep_close_down<DM>(P, sh, sg);
  const double* W = sh.W1;
  const double* A = sh.A;
  sep_reduce<DM>(P * DM * DM * DM, sh.part, out, [&](int o, int q) {   // q = (p, m, v, g)
    const int r = o / DM, ss = o % DM, g = q % DM, pmv = q / DM;
    return W[(pmv * DM + r) * DM + g] * A[(pmv * DM + ss) * DM + g];
  });
}

// f'[l][m] from the right half in W2 = sum_{p,v,s,g} (W2 sig)[p][l][v][s][g] A[p,m,v,s,g]
template <int DM>
__device__ void sep_f_from_right(int P, const SepSh& sh, const double* sg, double* out) {
  constexpr int V3 = DM * DM * DM;
  sep_close_down<DM>(P, sh, sg);
  const double* W = sh.W1;
  const double* A = sh.A;
  sep_reduce<DM>(P * V3, sh.part, out, [&](int o, int q) {   // q = (p, v, s, g)
    const int l = o / DM, m = o % DM, vsg = q % V3, p = q / V3;
    return W[(p * DM + l) * V3 + vsg] * A[(p * DM + m) * V3 + vsg];
  });
}

}  // namespace

template <int DM>
__global__ __launch_bounds__(SEP_T) void sep_kernel(const SepDesc* __restrict__ ds, int a_in_lds) {
  extern __shared__ double sep_lds[];
  constexpr int V4 = DM * DM * DM * DM, V2 = DM * DM;
  const SepDesc& D = ds[blockIdx.x];
  __shared__ double red[SEP_T / 64];
  __shared__ double one[SEP_V];
  __shared__ double part[SEP_T];
  __shared__ double mats[5 * SEP_V];
  const int P = D.sites[0].d;
  SepSh sh;
  sh.W1 = sep_lds;
  sh.W2 = sep_lds + 2 * V4;
  // the staged site: in LDS, or (DM = 8, where LDS holds only the two
  // intermediates) in the direction's global work buffer
  sh.A = a_in_lds ? sep_lds + 4 * V4 : D.work + (size_t)(3 * D.Lc + 3) * SEP_V;
  sh.part = part;
  sh.B = mats;
  sh.e = mats + SEP_V;
  sh.su = mats + 2 * SEP_V;
  sh.f = mats + 3 * SEP_V;
  sh.sg = mats + 4 * SEP_V;
  sh.red = red;
  const int Lr = D.Lr, Lc = D.Lc;
  double* E = D.work;                        // (Lc+1) padded slots
  double* F = E + (size_t)(Lc + 1) * SEP_V;  // (Lc+1) padded slots
  double* OLD = F + (size_t)(Lc + 1) * SEP_V;
  if (threadIdx.x < V2) {
    const double v = threadIdx.x == 0 ? 1.0 : 0.0;
    one[threadIdx.x] = v;
    E[threadIdx.x] = v;
    F[(size_t)Lc * SEP_V + threadIdx.x] = v;
  }
  __syncthreads();
  for (int k = 0; k + 1 < Lr; ++k) {
    const SepSite* row = D.sites + (size_t)k * Lc;
    auto sup = [&](int c) -> const double* { return k == 0 ? one : D.sig + D.off[(size_t)(k - 1) * Lc + c]; };
    auto sig = [&](int c) -> double* { return D.sig + D.off[(size_t)k * Lc + c]; };
    // sigma start: identity / sqrt(D) (compact Dd x Dd in global memory)
    for (int c = 0; c < Lc; ++c) {
      const int Dd = row[c].Dd;
      for (int i = threadIdx.x; i < Dd * Dd; i += SEP_T) sig(c)[i] = (i / Dd == i % Dd) ? 1.0 / sqrt((double)Dd) : 0.0;
    }
    __syncthreads();
    for (int c = Lc - 1; c >= 1; --c) {
      // k = 0: the up closing is the padded 1 x 1 identity (the up legs have dimension 1)
      sep_stage<DM>(row[c], sh, nullptr, k == 0 ? nullptr : sup(c), F + (size_t)(c + 1) * SEP_V, sig(c));
      if (k == 0 && threadIdx.x < V2) sh.su[threadIdx.x] = one[threadIdx.x];
      __syncthreads();
      sep_right<DM>(P, sh);
      sep_f_from_right<DM>(P, sh, sh.sg, F + (size_t)c * SEP_V);
      sep_unit(F + (size_t)c * SEP_V, V2, red);
    }
    int sweeps = 0;
    double delta = 0.0;
    while (true) {
      for (int c = 0; c < Lc; ++c)
        for (int i = threadIdx.x; i < row[c].Dd * row[c].Dd; i += SEP_T) OLD[(size_t)c * SEP_V + i] = sig(c)[i];
      __syncthreads();
      for (int pass = 0; pass < 2; ++pass) {
        const bool l2r = pass == 0;
        for (int s = 0; s < Lc; ++s) {
          const int c = l2r ? s : Lc - 1 - s;
          const int Dd = row[c].Dd;
          sep_stage<DM>(row[c], sh, E + (size_t)c * SEP_V, k == 0 ? nullptr : sup(c), F + (size_t)(c + 1) * SEP_V,
                        nullptr);
          if (k == 0 && threadIdx.x < V2) sh.su[threadIdx.x] = one[threadIdx.x];
          __syncthreads();
          if (l2r) {   // b, then the left environment of c+1
            sep_left<DM>(P, sh);
            sep_b_from_left<DM>(P, sh, sh.B);
          } else {     // b, then the right environment of c
            sep_right<DM>(P, sh);
            sep_b_from_right<DM>(P, sh, sh.B);
          }
          sep_unit(sh.B, V2, red);
          for (int i = threadIdx.x; i < Dd * Dd; i += SEP_T) sig(c)[i] = sh.B[(i / Dd) * DM + i % Dd];
          if (l2r && c + 1 < Lc) {
            sep_e_from_left<DM>(P, sh, sh.B, E + (size_t)(c + 1) * SEP_V);
            sep_unit(E + (size_t)(c + 1) * SEP_V, V2, red);
          }
          if (!l2r && c > 0) {
            sep_f_from_right<DM>(P, sh, sh.B, F + (size_t)c * SEP_V);
            sep_unit(F + (size_t)c * SEP_V, V2, red);
          }
        }
      }
      __syncthreads();
      ++sweeps;
      double dmax = 0.0;
      for (int c = 0; c < Lc; ++c) {
        const int Dd = row[c].Dd;
        double s = 0.0;
        for (int i = threadIdx.x; i < Dd * Dd; i += SEP_T) {
          const double x = sig(c)[i] - OLD[(size_t)c * SEP_V + i];
          s += x * x;
        }
        s = sep_block_sum(s, red);
        dmax = fmax(dmax, sqrt(s));
      }
      delta = dmax;
      if (delta <= D.tol || sweeps >= D.max_sweeps) break;
    }
    if (threadIdx.x == 0) {
      D.sweeps[k] = sweeps;
      D.delta[k] = delta;
    }
    __syncthreads();
  }
}

template <int DM>
static void sep_launch_dm(const SepDesc* d, int nd, hipStream_t s) {
  const int v4 = (int)sizeof(double) * 2 * DM * DM * DM * DM;   // one d <= 2 site-sized array
  const bool a_in_lds = 3 * v4 <= 136 * 1024;                   // W1, W2 and the site
  const int lds = a_in_lds ? 3 * v4 : 2 * v4;
  if (lds > 48 * 1024)
    PE_HIP(hipFuncSetAttribute((const void*)sep_kernel<DM>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  sep_kernel<DM><<<nd, SEP_T, lds, s>>>(d, a_in_lds ? 1 : 0);
}

void launch_sep(const SepDesc* d, int nd, int dmax, hipStream_t s) {
  if (nd <= 0) return;
  switch (dmax) {
    case 1: case 2: sep_launch_dm<2>(d, nd, s); break;
    case 3: sep_launch_dm<3>(d, nd, s); break;
    case 4: sep_launch_dm<4>(d, nd, s); break;
    case 5: sep_launch_dm<5>(d, nd, s); break;
    case 6: sep_launch_dm<6>(d, nd, s); break;
    case 7: sep_launch_dm<7>(d, nd, s); break;
    case 8: sep_launch_dm<8>(d, nd, s); break;
    default: throw Error(ST_UNSUPPORTED, "CU_0 boundaries support virtual bonds up to 8");
  }
  PE_HIP(hipGetLastError());
}

// ===========================================================================
// Fused two-row column step (see K2Desc).  1024 threads (16 waves) per
// workgroup, one workgroup per (descriptor, e); the workgroup runs the whole
// chain of the column step for x = 0..X-1: the top boundary absorbed into the
// incoming environment, the ket and bra layers of row 1 and of row 2, then
// the bottom boundary, accumulated over x in registers.  Wave w owns block
// o = w of row 1 (o = its incoming legs (L, M)) and of row 2 (o = row 1's
// outgoing legs (r, s)): everything a wave computes for its own block stays
// in its private LDS area and needs no barrier; only row 1's output, which
// row 2 reads across blocks, and the bottom boundary slab are shared; they
// are double-buffered, so one barrier per x suffices.  Every intermediate lives in LDS (row pitches padded
// against bank conflicts); HBM sees the incoming environment (read from L2
// by the workgroups of one descriptor, which share an XCD), the boundary and
// site tensors and the outgoing environment.  MFMA f64 16x16x4, issued as
// D = B^T A^T so that lanes 0..15 run along the rows; 16 waves with at most
// 128 registers each keep four waves on every SIMD.
// ===========================================================================
namespace {

constexpr int K2_T = 1024, K2_W = 16;
constexpr int K2_QP = 17;              // pitch of a [16][16] block (rows of 16 + 1)
constexpr int K2_BP = 16 * K2_QP;      // one such block
constexpr int K2_ZP = 33;              // pitch of the ket intermediate's rows
constexpr int K2_PRIV = 16 * K2_ZP;    // private LDS of one wave (doubles): its block, or its ket rows

__device__ inline d4_t k2_mma(double a, double b, d4_t c) {   // a: lane = (row, k); b: lane = (k, col)
  return __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c, 0, 0, 0);
}

__device__ inline d4_t k2_zero() {
  d4_t z;
  z[0] = z[1] = z[2] = z[3] = 0.0;
  return z;
}

// One row's ket and bra for one block, from the block's input In[q][k]
// (pitch K2_QP; q the bra's contracted leg pair, k the ket's):
//   Z[q][(ab,p)] = sum_k In[q][k] Ks[k][(ab,p)],  Y[ab][gs] = sum_(p,q) Z[q][(ab,p)] Bs[(p,q)][gs]
// Z (pitch K2_ZP) may share the wave's private area with In: the whole block
// is read into registers before Z is written.  Returns this lane's part of Y
// (rows ab = lane & 15, columns gs = lane / 16 + 4j).
// SW: In is an unpadded [16][16] block whose columns are XOR-swizzled per
// row (column k of row q at q*16 + (k ^ k2_swz(q))), else a padded one.
__device__ inline int k2_swz(int q) { return 4 * ((q >> 1) & 3); }

template <bool SW>
__device__ inline d4_t k2_row(const double* In, const double* Ks, const double* Bs, double* Z, int lr, int lk) {
  double av[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) av[s] = SW ? In[lr * 16 + ((4 * s + lk) ^ k2_swz(lr))] : In[lr * K2_QP + 4 * s + lk];
  d4_t z0 = k2_zero(), z1 = k2_zero();
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    z0 = k2_mma(av[s], Ks[(4 * s + lk) * 32 + lr], z0);
    z1 = k2_mma(av[s], Ks[(4 * s + lk) * 32 + 16 + lr], z1);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();   // In is read before Z overwrites it
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    Z[lr * K2_ZP + lk + 4 * j] = z0[j];
    Z[lr * K2_ZP + 16 + lk + 4 * j] = z1[j];
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // two accumulators (even and odd k steps), so that consecutive MFMAs do not depend on each other
  d4_t ya = k2_zero(), yb = k2_zero();
#pragma unroll
  for (int s = 0; s < 8; s += 2) {
    const int ka = 4 * s + lk, kb = ka + 4;
    const double za = Z[(ka & 15) * K2_ZP + lr * 2 + (ka >> 4)], ba = Bs[ka * 16 + lr];
    const double zb = Z[(kb & 15) * K2_ZP + lr * 2 + (kb >> 4)], bq = Bs[kb * 16 + lr];
    ya = k2_mma(za, ba, ya);
    yb = k2_mma(zb, bq, yb);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();   // Z is read before the area is rewritten
  return ya + yb;
}

}  // namespace

// Shared memory of one workgroup (CH: the launch's largest bond).
template <int CH>
struct K2Smem {
  double Te[CH * 16];
  double K1s[16 * 32], B1s[32 * 16], K2s[16 * 32], B2s[32 * 16];
  // shared, double-buffered by the parity of x: the bottom boundary slab and
  // row 1's output [(r,s)][(M,g)][(L,d)] (swizzled [16][16] blocks)
  double Bx[2][16 * CH];
  double Y2[2][16 * 256];
  double Priv[K2_W * K2_PRIV];   // per wave: its block or its ket rows
  int last;                      // this workgroup is the last slice of its output value
};

// One workgroup's column step (output value e of descriptor d, x slice sl).
// FULL: the descriptor's bonds a and y equal CH, so no partial tile is masked.
template <int CH, bool FULL>
__device__ __attribute__((always_inline)) inline void k2_body(const K2Desc& d, const int e, const int sl,
                                                              unsigned* counters, K2Smem<CH>& S) {
  static_assert(CH / 4 * K2_T == K2_PART || CH != K2_CHI, "partial result size");
  double* Te = S.Te;
  double *K1s = S.K1s, *B1s = S.B1s, *K2s = S.K2s, *B2s = S.B2s;
  double(*Bx)[16 * CH] = S.Bx;
  double(*Y2)[16 * 256] = S.Y2;
  double* Priv = S.Priv;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  double* Pw = Priv + w * K2_PRIV;
  const int X = d.X, A = FULL ? CH : d.A, Y = FULL ? CH : d.Y;
  const int A4 = FULL ? CH : (A + 3) & ~3;
  // ---- stage the site tensors and the top boundary column of this e
  for (int i = tid; i < 512; i += K2_T) {
    {   // K1s[(l,u)][(d,r,p)]
      const int k = i >> 5, n = i & 31, l = k >> 2, u = k & 3, dd = n >> 3, r = (n >> 1) & 3, p = n & 1;
      const int64_t* t = d.ss[0];
      K1s[i] = d.s[0][p * t[0] + l * t[1] + u * t[2] + r * t[3] + dd * t[4]];
    }
    {   // B1s[(p,(m,v))][(g,s)]
      const int row = i >> 4, col = i & 15, p = row >> 4, m = (row >> 2) & 3, vv = row & 3, g = col >> 2, sx = col & 3;
      const int64_t* t = d.ss[1];
      B1s[i] = d.s[1][p * t[0] + m * t[1] + vv * t[2] + sx * t[3] + g * t[4]];
    }
    {   // K2s[(L,d)][(D,R,q)]
      const int k = i >> 5, n = i & 31, L = k >> 2, dd = k & 3, D = n >> 3, R = (n >> 1) & 3, q = n & 1;
      const int64_t* t = d.ss[2];
      K2s[i] = d.s[2][q * t[0] + L * t[1] + dd * t[2] + R * t[3] + D * t[4]];
    }
    {   // B2s[(q,(M,g))][(G,S)]
      const int row = i >> 4, col = i & 15, q = row >> 4, M = (row >> 2) & 3, g = row & 3, G = col >> 2, S = col & 3;
      const int64_t* t = d.ss[3];
      B2s[i] = d.s[3][q * t[0] + M * t[1] + g * t[2] + S * t[3] + G * t[4]];
    }
  }
  for (int i = tid; i < A4 * 16; i += K2_T) {
    const int a = i >> 4, uv = i & 15;
    Te[i] = a < A ? d.T[a * d.sT[0] + (uv >> 2) * d.sT[1] + (uv & 3) * d.sT[2] + e * d.sT[3]] : 0.0;
  }
  const int nct = FULL ? CH / 16 : (Y + 15) >> 4;   // column tiles of the output
  d4_t out[CH / 16];
#pragma unroll
  for (int c = 0; c < CH / 16; ++c) out[c] = k2_zero();
  // This lane's row of the incoming environment (its row-1 block) and its
  // share of the bottom boundary slab; the values for x + 1 are loaded while
  // x is computed (each after its x values have gone to LDS).  Loads are
  // unconditional (indices clamped, values masked) so that they issue back
  // to back.
  // Per-lane element offsets (32-bit: a descriptor's tensors are far below
  // 2^31 elements), fixed over x; each x only moves the uniform base.
  const int ro = (int)((w >> 2) * d.sL[1] + (w & 3) * d.sL[2] + (lr >> 2) * d.sL[3] + (lr & 3) * d.sL[4]);   // (L,M,l,m)
  const int sa = (int)d.sL[5];
  constexpr int KMAX = CH / 4;
  constexpr int NBX = (16 * CH + K2_T - 1) / K2_T;
  int boff[NBX];
#pragma unroll
  for (int j = 0; j < NBX; ++j) {
    const int i = tid + K2_T * j, k = i / CH, y = i % CH, yc = y < Y ? y : Y - 1;
    boff[j] = (int)((k >> 2) * d.sB[1] + (k & 3) * d.sB[2] + yc * d.sB[3]);
  }
  double lxf[KMAX];
  double bxf[NBX];
  auto load_l = [&](int x) {
    const double* Lx = d.L + x * d.sL[0];
#pragma unroll
    for (int ks = 0; ks < KMAX; ++ks) {
      if (FULL) {
        lxf[ks] = Lx[ro + (4 * ks + lk) * sa];
      } else if (4 * ks < A4) {
        const int a = 4 * ks + lk, ac = a < A ? a : A - 1;
        const double val = Lx[ro + ac * sa];
        lxf[ks] = a < A ? val : 0.0;
      }
    }
  };
  auto load_b = [&](int x) {
    const double* Bx0 = d.B + x * d.sB[0];
#pragma unroll
    for (int j = 0; j < NBX; ++j) {
      const int i = tid + K2_T * j;
      if (i < 16 * CH) {
        const double val = Bx0[boff[j]];
        bxf[j] = (FULL || i % CH < Y) ? val : 0.0;
      }
    }
  };
  const int x0 = (int)((int64_t)sl * X / d.ns), x1 = (int)((int64_t)(sl + 1) * X / d.ns);
  if (x0 < x1) {
    load_l(x0);
    load_b(x0);
  }
  __syncthreads();

  for (int x = x0; x < x1; ++x) {
    // ---- row 1 for this wave's block o = (L, M): y1[(l,m)][(u,v)] = sum_a Lin[x,L,M,l,m,a] T[a,u,v,e]
    //      into the block [q=(m,v)][k=(l,u)], then ket and bra
    {
      d4_t acc = k2_zero(), acc2 = k2_zero();
#pragma unroll
      for (int ks = 0; ks < KMAX; ks += 2) {
        if (4 * ks < A4) acc = k2_mma(lxf[ks], Te[(4 * ks + lk) * 16 + lr], acc);
        if (4 * ks + 4 < A4) acc2 = k2_mma(lxf[ks + 1], Te[(4 * ks + 4 + lk) * 16 + lr], acc2);
      }
      acc += acc2;
      const int l = lr >> 2, m = lr & 3;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int uv = lk + 4 * j, u = uv >> 2, vv = uv & 3;
        Pw[(m * 4 + vv) * K2_QP + l * 4 + u] = acc[j];
      }
    }
    if (x + 1 < x1) load_l(x + 1);   // in flight during the rows and the bottom boundary
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const d4_t y2 = k2_row<false>(Pw, K1s, B1s, Pw, lr, lk);
    // row 1's output y2[(L,M)=w][(d,r)][(g,s)] -> Y2 [(r,s)][(M,g)][(L,d)]; the bottom slab of x.
    // The buffers of parity x & 1 were last read at x - 2, which every wave
    // finished before the barrier of x - 1, so no barrier is needed here.
    double* Y2x = Y2[x & 1];
    double* Bxx = Bx[x & 1];
    {
      const int L = w >> 2, M = w & 3, dd = lr >> 2, r = lr & 3;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int gs = lk + 4 * j, g = gs >> 2, sx = gs & 3, q2 = M * 4 + g;
        Y2x[(r * 4 + sx) * 256 + q2 * 16 + ((L * 4 + dd) ^ k2_swz(q2))] = y2[j];
      }
    }
#pragma unroll
    for (int j = 0; j < NBX; ++j)
      if (tid + K2_T * j < 16 * CH) Bxx[tid + K2_T * j] = bxf[j];
    if (x + 1 < x1) load_b(x + 1);   // in flight during row 2 and the bottom boundary
    __syncthreads();
    // ---- row 2 for this wave's block o = (r, s), then the bottom boundary:
    //      out[(r,s)][(R,S)][y] += sum_(D,G) y3[(r,s)][(R,S)][(D,G)] Bx[(D,G)][y]
    {
      const d4_t y3 = k2_row<true>(Y2x + w * 256, K2s, B2s, Pw, lr, lk);   // rows (D,R), columns (G,S)
      const int D = lr >> 2, R = lr & 3;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int GS = lk + 4 * j, G = GS >> 2, S = GS & 3;
        Pw[(R * 4 + S) * K2_QP + D * 4 + G] = y3[j];
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      double av[4], bv[4][CH / 16];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        av[s] = Pw[lr * K2_QP + 4 * s + lk];
#pragma unroll
        for (int c = 0; c < CH / 16; ++c) bv[s][c] = Bxx[(4 * s + lk) * CH + 16 * c + lr];
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < CH / 16; ++c)
          if (c < nct) out[c] = k2_mma(av[s], bv[s][c], out[c]);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();   // the block is read before the next x rewrites it
    }
  }
  // ---- x slices: this slice's partial result, device-scope stores (read by
  // whichever workgroup finishes the value last, on any XCD); the last one
  // sums the ns partials in slice order, so the result does not depend on
  // the order in which the slices finish.
  if (d.ns > 1) {
    int t1 = threadIdx.x;
    asm volatile("" : "+v"(t1));
    double* part = d.part + ((int64_t)e * d.ns + sl) * K2_PART;
#pragma unroll
    for (int c = 0; c < CH / 16; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        __hip_atomic_store(&part[(c * 4 + j) * K2_T + t1], out[c][j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);   // this thread's partial is complete before the counter moves
    __syncthreads();
    if (t1 == 0)
      S.last = __hip_atomic_fetch_add(counters + d.cnt_base + e, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
               (unsigned)(d.ns - 1);
    __syncthreads();
    if (!S.last) return;
    const double* tp = d.part + (int64_t)e * d.ns * K2_PART;
#pragma unroll
    for (int c = 0; c < CH / 16; ++c) out[c] = k2_zero();
    for (int q = 0; q < d.ns; ++q) {
      double v[CH / 16][4];
#pragma unroll
      for (int c = 0; c < CH / 16; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          v[c][j] = __hip_atomic_load(const_cast<double*>(&tp[(int64_t)q * K2_PART + (c * 4 + j) * K2_T + t1]),
                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
      for (int c = 0; c < CH / 16; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j) out[c][j] += v[c][j];
    }
  }
  // ---- store: this lane's rows (R,S) = lane & 15 of block (r,s) = w; columns y.
  // The lane index is re-read through an empty asm so that the store
  // addresses are formed here: hoisted above the x loop they would stay live
  // through it and spill.
  {
    int t2 = threadIdx.x;
    asm volatile("" : "+v"(t2));
    const int w2 = t2 >> 6, l2 = t2 & 63, lr2 = l2 & 15, lk2 = l2 >> 4;
    const int r = w2 >> 2, sx = w2 & 3, R = lr2 >> 2, S = lr2 & 3;
    const int64_t rowoff = R * d.sO[1] + S * d.sO[2] + r * d.sO[3] + sx * d.sO[4] + e * d.sO[5];
#pragma unroll
    for (int c = 0; c < CH / 16; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int y = 16 * c + lk2 + 4 * j;
        if (c < nct && y < Y) d.O[rowoff + y * d.sO[0]] = out[c][j];
      }
  }
}


template <int CH>
__global__ __launch_bounds__(K2_T) void k2_kernel(const K2Desc* __restrict__ ds, int nd, int nblocks,
                                                  unsigned* counters) {
  __shared__ K2Smem<CH> S;
  // XCD-aware order: consecutive virtual blocks (the e values of one
  // descriptor) go to one XCD, so they share the incoming environment in L2
  const int grid = gridDim.x, per = grid / 8;
  const int v = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (v >= nblocks) return;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ds[mid].block_base <= v) lo = mid; else hi = mid - 1;
  }
  const K2Desc& d = ds[lo];
  // slice-major within a descriptor: consecutive workgroups take the same x
  // slice of successive output values and share its rows of L in L2
  const int u = v - d.block_base, sl = u / d.E, e = u - sl * d.E;
  if (d.A == CH && d.Y == CH)
    k2_body<CH, true>(d, e, sl, counters, S);
  else
    k2_body<CH, false>(d, e, sl, counters, S);
}

// One-row chain step: wave w of a workgroup takes x = KC_W * xt + w for the
// workgroup's (xt, e); the top boundary slab of e and both sites are staged
// in LDS once per workgroup, the wave's row of E is read from global memory
// (shared by the Ne workgroups of one xt, which run on one XCD).
constexpr int KC_T = 64 * KC_W;   // threads per workgroup

__global__ __launch_bounds__(KC_T) void kc_kernel(const KcDesc* __restrict__ ds, int nd, int nblocks) {
  __shared__ double Te[K2_CHI * 16];
  __shared__ double Ks[16 * 32], Bs[32 * 16];
  __shared__ double Priv[KC_W * K2_PRIV];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  double* Pw = Priv + w * K2_PRIV;
  const int grid = gridDim.x, per = grid / 8;
  const int v = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (v >= nblocks) return;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ds[mid].block_base <= v) lo = mid; else hi = mid - 1;
  }
  const KcDesc& d = ds[lo];
  const int local = v - d.block_base, xq = local / d.Ne, e = local - xq * d.Ne;
  const int A = d.A, A4 = (A + 3) & ~3;
  for (int i = tid; i < 512; i += KC_T) {
    {   // Ks[(l,u)][(d,r,p)]
      const int k = i >> 5, n = i & 31, l = k >> 2, u = k & 3, dd = n >> 3, r = (n >> 1) & 3, p = n & 1;
      const int64_t* t = d.ss[0];
      Ks[i] = d.s[0][p * t[0] + l * t[1] + u * t[2] + r * t[3] + dd * t[4]];
    }
    {   // Bs[(p,(m,v))][(g,s)]
      const int row = i >> 4, col = i & 15, p = row >> 4, m = (row >> 2) & 3, vv = row & 3, g = col >> 2, sx = col & 3;
      const int64_t* t = d.ss[1];
      Bs[i] = d.s[1][p * t[0] + m * t[1] + vv * t[2] + sx * t[3] + g * t[4]];
    }
  }
  for (int i = tid; i < A4 * 16; i += KC_T) {
    const int a = i >> 4, uv = i & 15;
    Te[i] = a < A ? d.T[a * d.sT[0] + (uv >> 2) * d.sT[1] + (uv & 3) * d.sT[2] + e * d.sT[3]] : 0.0;
  }
  constexpr int KMAX = K2_CHI / 4;
  const int ngroups = (d.X + KC_W - 1) / KC_W;
  for (int r = 0; r < d.xr; ++r) {
    const int xt = xq * d.xr + r;
    if (xt >= ngroups) break;   // the same for every wave of the workgroup
    // this wave's x (clamped for the loads; waves past X store nothing) and
    // its lane's row (l, m) = lr of E, a = 4 ks + lk
    const int x = KC_W * xt + w;
    const bool act = x < d.X;
    const double* Ex = d.E + (act ? x : d.X - 1) * d.sE[0] + (lr >> 2) * d.sE[1] + (lr & 3) * d.sE[2];
    double lxf[KMAX];
#pragma unroll
    for (int ks = 0; ks < KMAX; ++ks) {
      if (4 * ks < A4) {
        const int a = 4 * ks + lk, ac = a < A ? a : A - 1;
        const double val = Ex[ac * d.sE[3]];
        lxf[ks] = a < A ? val : 0.0;
      }
    }
    if (r == 0) __syncthreads();   // the staged sites and slab
    // y1[(l,m)][(u,v)] = sum_a E[x,l,m,a] T[a,u,v,e] into the block [q=(m,v)][k=(l,u)]
    {
      d4_t acc = k2_zero(), acc2 = k2_zero();
#pragma unroll
      for (int ks = 0; ks < KMAX; ks += 2) {
        if (4 * ks < A4) acc = k2_mma(lxf[ks], Te[(4 * ks + lk) * 16 + lr], acc);
        if (4 * ks + 4 < A4) acc2 = k2_mma(lxf[ks + 1], Te[(4 * ks + 4 + lk) * 16 + lr], acc2);
      }
      acc += acc2;
      const int l = lr >> 2, m = lr & 3;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int uv = lk + 4 * j, u = uv >> 2, vv = uv & 3;
        Pw[(m * 4 + vv) * K2_QP + l * 4 + u] = acc[j];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const d4_t y2 = k2_row<false>(Pw, Ks, Bs, Pw, lr, lk);   // [(d,r)][(g,s)]
    if (act) {
      const int dd = lr >> 2, rr = lr & 3;
      const int64_t base = x * d.sY[0] + dd * d.sY[1] + rr * d.sY[3] + e * d.sY[5];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int gs = lk + 4 * j, g = gs >> 2, sx = gs & 3;
        d.Y[base + g * d.sY[2] + sx * d.sY[4]] = y2[j];
      }
    }
  }
}

void launch_kc(const KcDesc* d, int nd, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return;
  const int grid = (nblocks + 7) / 8 * 8;   // a multiple of the XCD count: the block order is a bijection
  kc_kernel<<<grid, KC_T, 0, s>>>(d, nd, nblocks);
  PE_HIP(hipGetLastError());
}

void launch_k2(const K2Desc* d, int nd, int nblocks, int chmax, unsigned* counters, hipStream_t s) {
  if (nblocks <= 0) return;
  const int grid = (nblocks + 7) / 8 * 8;   // a multiple of the XCD count: the block order is a bijection
  if (chmax > K2_CHI) throw Error(ST_INVALID, "two-row column step: bond above the fused kernel's limit");
  k2_kernel<K2_CHI><<<grid, K2_T, 0, s>>>(d, nd, nblocks, counters);
  PE_HIP(hipGetLastError());
}

}  // namespace pe
