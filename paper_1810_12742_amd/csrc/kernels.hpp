// Device code of the MI355X Hines solver (included once, by hines.hip).
//
// A group (packed cells, paper §4) is solved by one workgroup.  Its
// compartments form an "image": d, u, b per slot, held in LDS when it fits
// (staged from HBM by global->LDS DMA) or in a global workspace otherwise.
// Slots follow the user numbering of each cell (kLdsPad unused slots in front
// and behind), so a branch is a run of consecutive slots.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "setup.hpp"

namespace hdev {

using hines::KBranch;
using hines::KCell;
using hines::KGroup;
using hines::kLdsPad;
using hines::LdsLayout;

struct DevTables {
  const KBranch* br;     // per group: level order, or (lane, start) order when scheduled
  const KGroup* grp;
  const int32_t* seg;    // first record of each (group, level) segment
  const KCell* cell;     // group order
  const int32_t* glist;  // group ids of one launch
  const int32_t* lanes;  // scheduled plans: per group kSchedLanes + 1 record offsets
  double* ws;            // global images of groups that exceed LDS
  const KBranch* br_level;  // records in level order (same as br unless scheduled)
};

// Right-hand side of a solve: given (kRhsGiven), c v + i (kRhsCV; i may be
// absent), or c v + sigma Z(seed, step, user index) (kRhsNoise).
enum : int32_t { kRhsGiven = 0, kRhsCV = 1, kRhsNoise = 2 };
struct RhsSpec {
  const double* rhs;
  const double* c;
  const double* v;
  const double* icur;
  double sigma;
  uint32_t seed, step;
  int32_t mode, pad;
};

typedef __attribute__((address_space(3))) void lds_void_t;

// ---- Philox4x32-10 (Salmon et al., SC'11) and the Box-Muller draw ---------
__device__ __forceinline__ double noise_draw(uint32_t seed, uint32_t step, uint64_t i, double sigma) {
  uint32_t c0 = (uint32_t)i, c1 = (uint32_t)(i >> 32), c2 = step, c3 = 0u;
  uint32_t k0 = seed, k1 = 0u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  const uint64_t m1 = ((((uint64_t)c0) << 32) | c1) >> 12;
  const uint64_t m2 = ((((uint64_t)c2) << 32) | c3) >> 12;
  const double u1 = ((double)m1 + 0.5) * 0x1p-52;
  const double u2 = ((double)m2 + 0.5) * 0x1p-52;
  return sigma * (sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2));
}

__device__ __forceinline__ double rhs_value(const RhsSpec& rs, int64_t i) {
  double v = rs.c[i] * rs.v[i];
  if (rs.mode == kRhsNoise)
    v = v + noise_draw(rs.seed, rs.step, (uint64_t)i, rs.sigma);
  else if (rs.icur)
    v = v + rs.icur[i];
  return v;
}

// ---- bulk copies -------------------------------------------------------------
// 16-byte global->LDS DMA: each lane moves one 16-byte unit, a wave instruction
// moves 1 KiB; the LDS side is 16-byte aligned, the global side 8-byte.
template <int T>
__device__ __forceinline__ void dma16(const void* src, void* dst, int units, int tid) {
  constexpr int W = T / 64;
  const int lane = tid & 63;
  const char* s = (const char*)src;
  char* d = (char*)dst;
  for (int c = tid >> 6; c * 64 < units; c += W) {
    const int p = c * 64 + lane;
    if (p < units) __builtin_amdgcn_global_load_lds((const void*)(s + 16 * p), (lds_void_t*)(d + 1024 * c), 16, 0, 0);
  }
}

template <int T>
__device__ __forceinline__ void dma4(const void* src, void* dst, int units, int tid) {
  constexpr int W = T / 64;
  const int lane = tid & 63;
  const char* s = (const char*)src;
  char* d = (char*)dst;
  for (int c = tid >> 6; c * 64 < units; c += W) {
    const int p = c * 64 + lane;
    if (p < units) __builtin_amdgcn_global_load_lds((const void*)(s + 4 * p), (lds_void_t*)(d + 256 * c), 4, 0, 0);
  }
}

// Image slots [slot, slot + n) <- user range [lo, lo + n).  LDS images use
// DMA for the pairs (slot even) and registers for an odd last element; a
// global image is copied through registers.  A computed right-hand side is
// written through registers in both cases.
template <int T, bool GLOBAL>
__device__ __forceinline__ void stage_range(const RhsSpec& rs, const double* d, const double* u, int64_t lo, int n,
                                            int slot, double* D, double* U, double* B, int tid) {
  if constexpr (GLOBAL) {
#pragma unroll 4
    for (int k = tid; k < n; k += T) {
      D[slot + k] = d[lo + k];
      U[slot + k] = u[lo + k];
      B[slot + k] = rs.mode == kRhsGiven ? rs.rhs[lo + k] : rhs_value(rs, lo + k);
    }
  } else {
    const int units = n >> 1;
    dma16<T>(d + lo, D + slot, units, tid);
    dma16<T>(u + lo, U + slot, units, tid);
    if (rs.mode == kRhsGiven) {
      dma16<T>(rs.rhs + lo, B + slot, units, tid);
      if ((n & 1) && tid == 0) B[slot + n - 1] = rs.rhs[lo + n - 1];
    } else {
#pragma unroll 4
      for (int k = tid; k < n; k += T) B[slot + k] = rhs_value(rs, lo + k);
    }
    if ((n & 1) && tid == 0) {
      D[slot + n - 1] = d[lo + n - 1];
      U[slot + n - 1] = u[lo + n - 1];
    }
  }
}

template <int T, bool GLOBAL>
__device__ __forceinline__ void stage_group(const DevTables& tb, const KGroup& G, const LdsLayout& L,
                                            const RhsSpec& rs, const double* d, const double* u, double* D,
                                            double* U, double* B, char* lds, int tid,
                                            const int32_t* lane_table) {
  dma16<T>(tb.br + G.br_begin, lds + L.br_off_bytes(), G.nbr, tid);
  if (lane_table)
    dma4<T>(lane_table, lds + L.tab_off_bytes(), hines::kSchedLanes + 1, tid);
  else
    dma4<T>(tb.seg + G.seg_begin, lds + L.tab_off_bytes(), G.nlev + 1, tid);
  if (G.contig) {
    // slots kLdsPad + [0, user_lo + user_n) <-> user [user_base, ...)
    stage_range<T, GLOBAL>(rs, d, u, G.user_base, G.user_lo + G.user_n, kLdsPad, D, U, B, tid);
  } else {
    for (int c = 0; c < G.ncell; ++c) {
      const KCell C = tb.cell[G.cell_begin + c];
      stage_range<T, GLOBAL>(rs, d, u, C.user_lo, C.n, C.lds, D, U, B, tid);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);  // every DMA of this wave has landed
  __syncthreads();
}

template <int T>
__device__ __forceinline__ void store_range(const double* B, int slot, double* x, int64_t lo, int n, int tid) {
  const int units = n >> 1;
  const double2* src = (const double2*)(B + slot);
  double2* dst = (double2*)(x + lo);
#pragma unroll 4
  for (int k = tid; k < units; k += T) {
    const double2 v = src[k];
    dst[k] = v;
  }
  if ((n & 1) && tid == 0) x[lo + n - 1] = B[slot + n - 1];
}

template <int T>
__device__ __forceinline__ void store_group(const DevTables& tb, const KGroup& G, const double* B, double* x,
                                            int tid) {
  if (G.contig) {
    const int lo = G.user_lo, hi = G.user_lo + G.user_n;
    const int a = (lo + 1) & ~1;  // first even offset at or after lo
    const double* Bp = B + kLdsPad;
    if (lo < a && tid == 0) x[G.user_base + lo] = Bp[lo];
    if (hi > a) store_range<T>(Bp, a, x, G.user_base + a, hi - a, tid);
  } else {
    for (int c = 0; c < G.ncell; ++c) {
      const KCell C = tb.cell[G.cell_begin + c];
      store_range<T>(B, C.lds, x, C.user_lo, C.n, tid);
    }
  }
}

// Reciprocal: hardware estimate (about 2^-24 relative) refined by one
// second-order Newton step, r1 = r0 (1 + e + e^2) with e = 1 - d r0.
__device__ __forceinline__ double rcp_nr(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  const double e = __builtin_fma(-d, r, 1.0);
  const double t = __builtin_fma(e, e, e);
  return __builtin_fma(r, t, r);
}

constexpr int kChunk = hines::kSchedChunk;  // compartments held in registers per LDS round trip

// ---------------------------------------------------------------------------
// Sweeps of one branch (paper §2 Listing 2, §3).  Branch compartments p_0 (root
// side) ... p_{len-1}; u_j couples p_j to p_{j-1} (stored at p_j for a branch
// running toward higher user indices, at p_{j-1}, the old child, for one
// running toward lower ones after re-rooting).  The pull subtracts the
// children's contributions in descending order of their first user index.
//
// Fast form.  Backward: r_j = 1/d'_j, f_j = u_j r_j, y_j = b'_j r_j stored in
// place of d_j, b_j; d'_{j-1} = d_{j-1} - f_j u_j, b'_{j-1} = b_{j-1} - f_j b'_j;
// at j = 0 the root stores x = b' r, any other branch its contribution
// (f_0 u_0, f_0 b'_0) in its own slot.  Forward: x_j = y_j - f_j x_{j-1}.
// Bitwise form: the plain algorithm's IEEE divisions and separately rounded
// multiply-subtract, in its order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void backward_fast(const KBranch br, double* D, const double* U, double* B, double* CD,
                                              double* CB) {
  const int dir = br.lendir > 0 ? 1 : -1;
  const int len = br.lendir > 0 ? br.lendir : -br.lendir;
  const int uoff = dir > 0 ? 0 : 1;
  int i = br.start + dir * (len - 1);
  double dl = D[i], bl = B[i];
  for (int k = br.nchild - 1; k >= 0; --k) {
    dl = dl - CD[br.child0 + k];
    bl = bl - CB[br.child0 + k];
  }
  int j = len - 1;
  while (j > 0) {
    const int n = j < kChunk ? j : kChunk;
    double uu[kChunk], dm[kChunk], bm[kChunk];
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      if (k < n) {
        const int ik = i - dir * k;
        uu[k] = U[ik + uoff];
        dm[k] = D[ik - dir];
        bm[k] = B[ik - dir];
      }
    }
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      if (k < n) {
        const double r = rcp_nr(dl);
        const double f = uu[k] * r;
        D[i] = f;
        B[i] = bl * r;
        dl = __builtin_fma(-f, uu[k], dm[k]);
        bl = __builtin_fma(-f, bl, bm[k]);
        i -= dir;
      }
    }
    j -= n;
  }
  const double r = rcp_nr(dl);
  if (br.u0 >= 0) {
    const double uu = U[br.u0];
    const double f = uu * r;
    D[i] = f;
    B[i] = bl * r;
    CD[br.self] = f * uu;
    CB[br.self] = f * bl;
  } else {
    B[i] = bl * r;
  }
}

__device__ __forceinline__ void forward_fast(const KBranch br, const double* D, double* B) {
  const int dir = br.lendir > 0 ? 1 : -1;
  const int len = br.lendir > 0 ? br.lendir : -br.lendir;
  int i = br.start;
  double xp;
  if (br.u0 >= 0) {
    xp = __builtin_fma(-D[i], B[br.pslot], B[i]);
    B[i] = xp;
  } else {
    xp = B[i];
  }
  int j = 1;
  while (j < len) {
    const int n = (len - j) < kChunk ? (len - j) : kChunk;
    double ff[kChunk], yy[kChunk];
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      if (k < n) {
        ff[k] = D[i + dir * (k + 1)];
        yy[k] = B[i + dir * (k + 1)];
      }
    }
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      if (k < n) {
        i += dir;
        xp = __builtin_fma(-ff[k], xp, yy[k]);
        B[i] = xp;
      }
    }
    j += n;
  }
}

// One chunk (up to kChunk steps) of the backward sweep of an ascending branch
// from slot i; the window may read up to kChunk slots below the branch (the
// padding or other branches) but writes only inside it.
__device__ __forceinline__ void backward_chunk_asc(int& i, int n, double& dl, double& bl, double* D, const double* U,
                                                   double* B) {
  const double* pd = D + (i - kChunk);  // pd[8-k] = D[i-k], pd[7-k] = D[i-k-1]
  const double* pu = U + (i - kChunk);
  const double* pb = B + (i - kChunk);
  double uu[kChunk], dm[kChunk], bm[kChunk], ff[kChunk], yy[kChunk];
#pragma unroll
  for (int k = 0; k < kChunk; ++k) {
    uu[k] = pu[kChunk - k];
    dm[k] = pd[kChunk - 1 - k];
    bm[k] = pb[kChunk - 1 - k];
  }
#pragma unroll
  for (int k = 0; k < kChunk; ++k) {
    if (k < n) {
      const double r = rcp_nr(dl);
      ff[k] = uu[k] * r;
      yy[k] = bl * r;
      dl = __builtin_fma(-ff[k], uu[k], dm[k]);
      bl = __builtin_fma(-ff[k], bl, bm[k]);
    }
  }
  double* qd = D + (i - kChunk);
  double* qb = B + (i - kChunk);
#pragma unroll
  for (int k = 0; k < kChunk; ++k) {
    if (k < n) {
      qd[kChunk - k] = ff[k];
      qb[kChunk - k] = yy[k];
    }
  }
  i -= n;
}

// One chunk of the forward sweep of an ascending branch after slot i; the
// window may read up to kChunk slots above the branch.
__device__ __forceinline__ void forward_chunk_asc(int& i, int n, double& xp, const double* D, double* B) {
  const double* pd = D + (i + 1);
  double* pb = B + (i + 1);
  double ff[kChunk], yy[kChunk], xs[kChunk];
#pragma unroll
  for (int k = 0; k < kChunk; ++k) {
    ff[k] = pd[k];
    yy[k] = pb[k];
  }
#pragma unroll
  for (int k = 0; k < kChunk; ++k) {
    if (k < n) {
      xp = __builtin_fma(-ff[k], xp, yy[k]);
      xs[k] = xp;
    }
  }
#pragma unroll
  for (int k = 0; k < kChunk; ++k)
    if (k < n) pb[k] = xs[k];
  i += n;
}

__device__ __forceinline__ void finish_backward(const KBranch br, int i, double dl, double bl, double* D,
                                                const double* U, double* B, double* CD, double* CB) {
  const double r = rcp_nr(dl);
  if (br.u0 >= 0) {
    const double uu = U[br.u0];
    const double f = uu * r;
    D[i] = f;
    B[i] = bl * r;
    CD[br.self] = f * uu;
    CB[br.self] = f * bl;
  } else {
    B[i] = bl * r;
  }
}

__device__ __forceinline__ void backward_asc(const KBranch br, double* D, const double* U, double* B, double* CD,
                                             double* CB) {
  const int len = br.lendir;
  int i = br.start + len - 1;
  double dl = D[i], bl = B[i];
  for (int k = br.nchild - 1; k >= 0; --k) {
    dl = dl - CD[br.child0 + k];
    bl = bl - CB[br.child0 + k];
  }
  for (int rem = len - 1; rem > 0;) {
    const int n = rem < kChunk ? rem : kChunk;
    backward_chunk_asc(i, n, dl, bl, D, U, B);
    rem -= n;
  }
  finish_backward(br, i, dl, bl, D, U, B, CD, CB);
}

__device__ __forceinline__ void forward_asc(const KBranch br, const double* D, double* B) {
  int i = br.start;
  double xp;
  if (br.u0 >= 0) {
    xp = __builtin_fma(-D[i], B[br.pslot], B[i]);
    B[i] = xp;
  } else {
    xp = B[i];
  }
  for (int rem = br.lendir - 1; rem > 0;) {
    const int n = rem < kChunk ? rem : kChunk;
    forward_chunk_asc(i, n, xp, D, B);
    rem -= n;
  }
}

__device__ __forceinline__ void backward_bitwise(const KBranch br, double* D, const double* U, double* B, double* CD,
                                                 double* CB) {
#pragma clang fp contract(off)
  const int dir = br.lendir > 0 ? 1 : -1;
  const int len = br.lendir > 0 ? br.lendir : -br.lendir;
  const int uoff = dir > 0 ? 0 : 1;
  int i = br.start + dir * (len - 1);
  double dl = D[i], bl = B[i];
  for (int k = br.nchild - 1; k >= 0; --k) {
    dl = dl - CD[br.child0 + k];
    bl = bl - CB[br.child0 + k];
  }
  for (int j = len - 1; j >= 1; --j) {
    const double uu = U[i + uoff];
    const double f = uu / dl;
    const int im = i - dir;
    const double dn = D[im] - f * uu;
    const double bn = B[im] - f * bl;
    D[i] = dl;
    B[i] = bl;
    dl = dn;
    bl = bn;
    i = im;
  }
  D[i] = dl;
  if (br.u0 >= 0) {
    const double uu = U[br.u0];
    const double f = uu / dl;
    B[i] = bl;
    CD[br.self] = f * uu;
    CB[br.self] = f * bl;
  } else {
    B[i] = bl / dl;
  }
}

__device__ __forceinline__ void forward_bitwise(const KBranch br, const double* D, const double* U, double* B) {
#pragma clang fp contract(off)
  const int dir = br.lendir > 0 ? 1 : -1;
  const int len = br.lendir > 0 ? br.lendir : -br.lendir;
  const int uoff = dir > 0 ? 0 : 1;
  int i = br.start;
  double xp;
  if (br.u0 >= 0) {
    xp = (B[i] - U[br.u0] * B[br.pslot]) / D[i];
    B[i] = xp;
  } else {
    xp = B[i];
  }
  for (int j = 1; j < len; ++j) {
    i += dir;
    xp = (B[i] - U[i + uoff] * xp) / D[i];
    B[i] = xp;
  }
}

enum { kModeFast = 0, kModeBitwise = 1, kModeAscending = 2 };

template <int MODE>
__device__ __forceinline__ void backward_branch(const KBranch br, double* D, const double* U, double* B, double* CD,
                                                double* CB) {
  if constexpr (MODE == kModeBitwise)
    backward_bitwise(br, D, U, B, CD, CB);
  else if constexpr (MODE == kModeAscending)
    backward_asc(br, D, U, B, CD, CB);
  else
    backward_fast(br, D, U, B, CD, CB);
}

template <int MODE>
__device__ __forceinline__ void forward_branch(const KBranch br, const double* D, const double* U, double* B) {
  if constexpr (MODE == kModeBitwise)
    forward_bitwise(br, D, U, B);
  else if constexpr (MODE == kModeAscending)
    forward_asc(br, D, B);
  else
    forward_fast(br, D, B);
}

// ---------------------------------------------------------------------------
// Level-synchronous solve (paper §3): levels deepest -> 0 for the backward
// sweep and 0 -> deepest for the forward sweep, a barrier between levels; lane
// t of the group takes branches t, t + T, ... of a level.  The first record
// of the next level is fetched while the current one runs.
// ---------------------------------------------------------------------------
template <int T, int MODE, bool GLOBAL>
__global__ __launch_bounds__(T) void k_solve_level(DevTables tb, RhsSpec rs, const double* __restrict__ d,
                                                   const double* __restrict__ u, double* x) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  const int g = tb.glist[blockIdx.x];
  const KGroup G = tb.grp[g];
  const LdsLayout L{GLOBAL ? 0 : G.nunk, (G.nbr + 1) & ~1, G.nlev};
  double* D = GLOBAL ? tb.ws + G.ws_off : (double*)lds_raw;
  double* U = D + G.nunk;
  double* B = D + 2 * (int64_t)G.nunk;
  double* CD = (double*)lds_raw + L.cd_off();
  double* CB = (double*)lds_raw + L.cb_off();
  const KBranch* BR = (const KBranch*)(lds_raw + L.br_off_bytes());
  const int* seg = (const int*)(lds_raw + L.tab_off_bytes());
  const int tid = threadIdx.x;
  const int brb = G.br_begin;

  stage_group<T, GLOBAL>(tb, G, L, rs, d, u, D, U, B, lds_raw, tid, nullptr);

  int s1 = seg[G.nlev] - brb;
  int s0 = seg[G.nlev - 1] - brb;
  KBranch cur{};
  if (s0 + tid < s1) cur = BR[s0 + tid];
  for (int l = G.nlev - 1; l >= 0; --l) {
    int p0 = 0;
    KBranch nxt{};
    if (l > 0) {
      p0 = seg[l - 1] - brb;
      if (p0 + tid < s0) nxt = BR[p0 + tid];
    }
    if (s0 + tid < s1) backward_branch<MODE>(cur, D, U, B, CD, CB);
    for (int e = s0 + tid + T; e < s1; e += T) backward_branch<MODE>(BR[e], D, U, B, CD, CB);
    __syncthreads();
    s1 = s0;
    s0 = p0;
    cur = nxt;
  }

  s0 = 0;
  s1 = seg[1] - brb;
  if (s0 + tid < s1) cur = BR[s0 + tid];
  for (int l = 0; l < G.nlev; ++l) {
    int p1 = 0;
    KBranch nxt{};
    if (l + 1 < G.nlev) {
      p1 = seg[l + 2] - brb;
      if (s1 + tid < p1) nxt = BR[s1 + tid];
    }
    if (s0 + tid < s1) forward_branch<MODE>(cur, D, U, B);
    for (int e = s0 + tid + T; e < s1; e += T) forward_branch<MODE>(BR[e], D, U, B);
    __syncthreads();
    s0 = s1;
    s1 = p1;
    cur = nxt;
  }

  store_group<T>(tb, G, B, x, tid);
}

// ---------------------------------------------------------------------------
// Scheduled solve (ascending branches, fast form, image in LDS).  One wave
// per group; lane t runs the branches the setup assigned to it, each from its
// scheduled iteration on; in one iteration a lane eliminates up to kChunk
// compartments of its current branch.  A branch starts only after every child
// branch finished in an earlier iteration, so the children's contributions
// are in LDS.  The forward sweep replays the schedule backwards in time: a
// branch's parent compartment is solved in a later backward iteration, hence
// in an earlier forward one.  The group is one wave and the LDS executes a
// wave's operations in order, so no barrier is needed between iterations; the
// signal fence keeps the compiler from moving LDS accesses across iterations.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int sched_itlen(int len) {
  const int k = (len - 1 + kChunk - 1) / kChunk;
  return k > 1 ? k : 1;
}

__global__ __launch_bounds__(64) void k_solve_sched(DevTables tb, RhsSpec rs, const double* __restrict__ d,
                                                    const double* __restrict__ u, double* x) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  const int g = tb.glist[blockIdx.x];
  const KGroup G = tb.grp[g];
  const LdsLayout L{G.nunk, (G.nbr + 1) & ~1, G.nlev};
  double* D = (double*)lds_raw;
  double* U = D + L.u_off();
  double* B = D + L.b_off();
  double* CD = D + L.cd_off();
  double* CB = D + L.cb_off();
  const KBranch* BR = (const KBranch*)(lds_raw + L.br_off_bytes());
  const int* LO = (const int*)(lds_raw + L.tab_off_bytes());
  const int lane = threadIdx.x;

  stage_group<64, false>(tb, G, L, rs, d, u, D, U, B, lds_raw, lane,
                         tb.lanes + (int64_t)g * (hines::kSchedLanes + 1));

  const int q0 = LO[lane], q1 = LO[lane + 1];
  const int F = G.makespan;
  {
    int q = q0, js = 0x7fffffff, i = 0, rem = -1;
    KBranch rec{};
    if (q < q1) {
      rec = BR[q];
      js = rec.pad;
    }
    double dl = 0.0, bl = 0.0;
    for (int it = 0; it < F; ++it) {
      if (q < q1 && it >= js) {
        if (it == js) {
          i = rec.start + rec.lendir - 1;
          dl = D[i];
          bl = B[i];
          for (int k = rec.nchild - 1; k >= 0; --k) {
            dl = dl - CD[rec.child0 + k];
            bl = bl - CB[rec.child0 + k];
          }
          rem = rec.lendir - 1;
        }
        if (rem > 0) {
          const int n = rem < kChunk ? rem : kChunk;
          backward_chunk_asc(i, n, dl, bl, D, U, B);
          rem -= n;
        }
        if (rem == 0) {
          finish_backward(rec, i, dl, bl, D, U, B, CD, CB);
          ++q;
          rem = -1;
          if (q < q1) {
            rec = BR[q];
            js = rec.pad;
          }
        }
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
  }
  __syncthreads();
  {
    int q = q1 - 1, je = -1, i = 0, rem = -1;
    KBranch rec{};
    if (q >= q0) {
      rec = BR[q];
      je = rec.pad + sched_itlen(rec.lendir) - 1;
    }
    double xp = 0.0;
    for (int it = F - 1; it >= 0; --it) {
      if (q >= q0 && it <= je) {
        if (it == je) {
          i = rec.start;
          if (rec.u0 >= 0) {
            xp = __builtin_fma(-D[i], B[rec.pslot], B[i]);
            B[i] = xp;
          } else {
            xp = B[i];
          }
          rem = rec.lendir - 1;
        }
        if (rem > 0) {
          const int n = rem < kChunk ? rem : kChunk;
          forward_chunk_asc(i, n, xp, D, B);
          rem -= n;
        }
        if (rem == 0) {
          --q;
          rem = -1;
          if (q >= q0) {
            rec = BR[q];
            je = rec.pad + sched_itlen(rec.lendir) - 1;
          }
        }
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
  }
  __syncthreads();
  store_group<64>(tb, G, B, x, lane);
}

// ---------------------------------------------------------------------------
// FP32 storage with FP64 refinement.  The matrix is the FP32 one (diag32,
// upper32), widened exactly where FP64 is used.  In LDS: d32, u32, f32 and a
// FP32 work vector w (4 bytes each), the FP64 rhs b and solution x.
//   sweep 0:  w = fl32(b); solve32(w); x = w
//   sweep s:  r = b - A x (FP64); w = fl32(r); solve32(w); x += w
// solve32 is the fast form of the sweeps in FP32 (level-synchronous).  The
// residual pulls each branch's children's couplings u_c x_c through the
// contribution slots, so every row is summed in a fixed order.
// ---------------------------------------------------------------------------
struct MixedLayout {
  int32_t nimg, nbr_pad, nlev;
  // floats d32, u32, f32, w at 0, nimg, 2 nimg, 3 nimg; doubles b, x after
  constexpr int64_t b_off_bytes() const { return 16 * (int64_t)nimg; }
  constexpr int64_t x_off_bytes() const { return 24 * (int64_t)nimg; }
  constexpr int64_t c_off_bytes() const { return 32 * (int64_t)nimg; }  // 2 nbr_pad doubles
  constexpr int64_t br_off_bytes() const { return c_off_bytes() + 16 * (int64_t)nbr_pad; }
  constexpr int64_t tab_off_bytes() const { return br_off_bytes() + 16 * (int64_t)nbr_pad; }
  constexpr int64_t bytes() const {
    const int64_t ints = (int64_t)nlev + 1;
    return (tab_off_bytes() + 4 * ints + 15) & ~(int64_t)15;
  }
};
__host__ __device__ constexpr MixedLayout mixed_layout(const KGroup& g) {
  return MixedLayout{g.nunk, (g.nbr + 1) & ~1, g.nlev};
}

template <int T>
__device__ __forceinline__ void stage_mixed_range(const float* d32, const float* u32, const double* b, int64_t lo,
                                                  int n, int slot, float* D, float* U, double* B, int tid) {
  dma4<T>(d32 + lo, D + slot, n, tid);
  dma4<T>(u32 + lo, U + slot, n, tid);
  dma16<T>(b + lo, B + slot, n >> 1, tid);
  if ((n & 1) && tid == 0) B[slot + n - 1] = b[lo + n - 1];
}

// One FP32 solve of A32 w' = w in place (generic branch direction).
template <int T>
__device__ __forceinline__ void solve32_level(const KBranch* BR, const int* seg, int brb, int nlev, const float* D,
                                              const float* U, float* F, float* W, float* CD, float* CB, int tid) {
  for (int l = nlev - 1; l >= 0; --l) {
    for (int e = seg[l] - brb + tid; e < seg[l + 1] - brb; e += T) {
      const KBranch br = BR[e];
      const int dir = br.lendir > 0 ? 1 : -1;
      const int len = br.lendir > 0 ? br.lendir : -br.lendir;
      const int uoff = dir > 0 ? 0 : 1;
      int i = br.start + dir * (len - 1);
      float dl = D[i], bl = W[i];
      for (int k = br.nchild - 1; k >= 0; --k) {
        dl = dl - CD[br.child0 + k];
        bl = bl - CB[br.child0 + k];
      }
      for (int j = len - 1; j >= 1; --j) {
        const float uu = U[i + uoff];
        const float r = __builtin_amdgcn_rcpf(dl);
        const float f = uu * r;
        F[i] = f;
        W[i] = bl * r;
        dl = __builtin_fmaf(-f, uu, D[i - dir]);
        bl = __builtin_fmaf(-f, bl, W[i - dir]);
        i -= dir;
      }
      const float r = __builtin_amdgcn_rcpf(dl);
      if (br.u0 >= 0) {
        const float uu = U[br.u0];
        const float f = uu * r;
        F[i] = f;
        W[i] = bl * r;
        CD[br.self] = f * uu;
        CB[br.self] = f * bl;
      } else {
        W[i] = bl * r;
      }
    }
    __syncthreads();
  }
  for (int l = 0; l < nlev; ++l) {
    for (int e = seg[l] - brb + tid; e < seg[l + 1] - brb; e += T) {
      const KBranch br = BR[e];
      const int dir = br.lendir > 0 ? 1 : -1;
      const int len = br.lendir > 0 ? br.lendir : -br.lendir;
      int i = br.start;
      float xp;
      if (br.u0 >= 0) {
        xp = __builtin_fmaf(-F[i], W[br.pslot], W[i]);
        W[i] = xp;
      } else {
        xp = W[i];
      }
      for (int j = 1; j < len; ++j) {
        i += dir;
        xp = __builtin_fmaf(-F[i], xp, W[i]);
        W[i] = xp;
      }
    }
    __syncthreads();
  }
}

// w = fl32(b - A x) over every compartment of the group.
template <int T>
__device__ __forceinline__ void residual_mixed(const KBranch* BR, int nbr, const float* D, const float* U,
                                               const double* B, const double* X, float* W, double* C, int tid) {
  for (int e = tid; e < nbr; e += T) {
    const KBranch br = BR[e];
    if (br.u0 >= 0) C[br.self] = (double)U[br.u0] * X[br.start];
  }
  __syncthreads();
  for (int e = tid; e < nbr; e += T) {
    const KBranch br = BR[e];
    const int dir = br.lendir > 0 ? 1 : -1;
    const int len = br.lendir > 0 ? br.lendir : -br.lendir;
    const int uoff = dir > 0 ? 0 : 1;
    int i = br.start;
    for (int j = 0; j < len; ++j, i += dir) {
      double r = B[i] - (double)D[i] * X[i];
      if (j > 0)
        r = r - (double)U[i + uoff] * X[i - dir];
      else if (br.u0 >= 0)
        r = r - (double)U[br.u0] * X[br.pslot];
      if (j < len - 1) {
        r = r - (double)U[i + dir + uoff] * X[i + dir];
      } else {
        for (int k = br.nchild - 1; k >= 0; --k) r = r - C[br.child0 + k];
      }
      W[i] = (float)r;
    }
  }
  __syncthreads();
}

template <int T>
__global__ __launch_bounds__(T) void k_solve_mixed(DevTables tb, const float* __restrict__ d32,
                                                   const float* __restrict__ u32, const double* b, double* x,
                                                   int sweeps) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  const int g = tb.glist[blockIdx.x];
  const KGroup G = tb.grp[g];
  const MixedLayout L = mixed_layout(G);
  float* D = (float*)lds_raw;
  float* U = D + L.nimg;
  float* F = D + 2 * (int64_t)L.nimg;
  float* W = D + 3 * (int64_t)L.nimg;
  double* B = (double*)(lds_raw + L.b_off_bytes());
  double* X = (double*)(lds_raw + L.x_off_bytes());
  double* C = (double*)(lds_raw + L.c_off_bytes());
  float* CD = (float*)C;
  float* CB = CD + L.nbr_pad;
  const KBranch* BR = (const KBranch*)(lds_raw + L.br_off_bytes());
  int* seg = (int*)(lds_raw + L.tab_off_bytes());
  const int tid = threadIdx.x;

  dma16<T>(tb.br_level + G.br_begin, lds_raw + L.br_off_bytes(), G.nbr, tid);
  dma4<T>(tb.seg + G.seg_begin, seg, G.nlev + 1, tid);
  if (G.contig) {
    stage_mixed_range<T>(d32, u32, b, G.user_base, G.user_lo + G.user_n, kLdsPad, D, U, B, tid);
  } else {
    for (int c = 0; c < G.ncell; ++c) {
      const KCell Cc = tb.cell[G.cell_begin + c];
      stage_mixed_range<T>(d32, u32, b, Cc.user_lo, Cc.n, Cc.lds, D, U, B, tid);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int k = tid; k < L.nimg; k += T) W[k] = (float)B[k];
  __syncthreads();
  const int brb = G.br_begin;
  for (int s = 0; s <= sweeps; ++s) {
    solve32_level<T>(BR, seg, brb, G.nlev, D, U, F, W, CD, CB, tid);
    for (int k = tid; k < L.nimg; k += T) X[k] = (s == 0 ? 0.0 : X[k]) + (double)W[k];
    __syncthreads();
    if (s < sweeps) residual_mixed<T>(BR, G.nbr, D, U, B, X, W, C, tid);
  }
  store_group<T>(tb, G, X, x, tid);
}

// ---------------------------------------------------------------------------
// Element-wise kernels of the time loop's adjoint (paper §1: A = diag(c) + L(a),
// symmetric).  All use the user numbering; children lists are CSR in
// ascending child index, so sums run in a fixed order.
// ---------------------------------------------------------------------------
// diag_i = c_i + a_i + sum over children k of a_k; upper_i = -a_i (0 at roots).
__global__ void k_assemble(int64_t n, const int32_t* __restrict__ parent, const int32_t* __restrict__ ch_off,
                           const int32_t* __restrict__ ch, const double* __restrict__ a,
                           const double* __restrict__ c, double* __restrict__ diag, double* __restrict__ upper) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool root = parent[i] < 0;
  double s = c[i];
  if (!root) s = s + a[i];
  for (int32_t e = ch_off[i]; e < ch_off[i + 1]; ++e) s = s + a[ch[e]];
  diag[i] = s;
  upper[i] = root ? 0.0 : -a[i];
}

// mu = c * lam_next, plus g[cell] at each cell's root.
__global__ void k_adjoint_rhs(int64_t n, const int32_t* __restrict__ parent, const int64_t* __restrict__ cell_off,
                              int32_t ncells, const double* __restrict__ c, const double* __restrict__ lam_next,
                              const double* __restrict__ g, double* __restrict__ mu) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double m = lam_next ? c[i] * lam_next[i] : 0.0;
  if (parent[i] < 0) {
    int32_t lo = 0, hi = ncells;  // the cell whose first compartment is i
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (cell_off[mid] <= i) lo = mid; else hi = mid;
    }
    m = m + g[lo];
  }
  mu[i] = m;
}

// out[cell] = v[first compartment of cell]
__global__ void k_gather_roots(int32_t ncells, const int64_t* __restrict__ cell_off, const double* __restrict__ v,
                               double* __restrict__ out) {
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  out[c] = v[cell_off[c]];
}

// Per step k: gI += lam; gc += lam (v_prev - v); ga_i += -(lam_i - lam_p)(v_i - v_p).
__global__ void k_adjoint_accumulate(int64_t n, const int32_t* __restrict__ parent, const double* __restrict__ lam,
                                     const double* __restrict__ v, const double* __restrict__ v_prev,
                                     double* __restrict__ ga, double* __restrict__ gc, double* __restrict__ gi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double l = lam[i];
  gi[i] = gi[i] + l;
  gc[i] = gc[i] + l * (v_prev[i] - v[i]);
  const int32_t p = parent[i];
  if (p >= 0) ga[i] = ga[i] - (l - lam[p]) * (v[i] - v[p]);
}

}  // namespace hdev
