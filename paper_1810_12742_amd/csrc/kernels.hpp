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
  const KBranch* br;     // per group, level order
  const KGroup* grp;
  const int32_t* seg;    // first record of each (group, level) segment
  const KCell* cell;     // group order
  const int32_t* glist;  // group ids of one launch
  double* ws;            // global images of groups that exceed LDS
  const hines::KFlow* flow;  // flow kernel: per group
  const uint64_t* fmask;     // flow kernel: active and push masks per step
  const uint16_t* fpos;      // flow kernel: position of every element
  const int16_t* faux;       // flow kernel: parent position of every push
  const hines::KCellWave* cwave;  // cell-lane kernel: per wave
  const int64_t* cbase;           // cell-lane kernel: first user index of each lane's cell
  const uint16_t* cpos;           // cell-lane kernel: positions, staging order
  const uint8_t* cflag;           // cell-lane kernel: flags, cell-lane order
  const uint64_t* cmsrc;          // cell-lane kernel: mailbox source lists per lane
  const uint64_t* crange;         // cell-lane kernel: per lane the steps [q0, q1) that are not padding
  double* czero;                  // cell-lane kernel: 1 KiB of zeros (64 lanes x 16 bytes), the stand-in
                                  // for walk-layout pairs of padding steps (only zeros are stored to it)
  double* cscr;                   // cell-lane kernels: (f, y) per step and lane
  int64_t cslots;                 // cell-lane kernel: steps x lanes of all waves (walk-layout array length)
  const hines::KCellWave* swave;  // index-order cell lanes: per wave
  const int64_t* sbase;           // index-order cell lanes: first user index of each lane's cell
  const uint16_t* spos;           // index-order cell lanes: positions, staging order
  const uint16_t* scode;          // index-order cell lanes: step codes, cell-lane order
  const uint64_t* smsrc;          // index-order cell lanes: mailbox source lists per lane
  const hines::KResGroup* rgrp;   // resident kernel: per group
  const int32_t* rlist;           // resident kernel: group ids of one launch
  const uint8_t* rblob;           // resident kernel: per-group lane offsets, roots and path records
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
    // one 32 x 32 -> 64-bit product per multiplier (high and low halves together)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
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
  // cos(2 pi u2) as cospi(2 u2): 2 u2 is exact, and the reduction by whole
  // periods is exact too (no multi-word reduction of a rounded 2 pi u2)
  return sigma * (sqrt(-2.0 * log(u1)) * cospi(2.0 * u2));
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
                                            double* U, double* B, char* lds, int tid) {
  dma16<T>(tb.br + G.br_begin, lds + L.br_off_bytes(), G.nbr, tid);
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

constexpr int kChunk = 8;  // compartments held in registers per LDS round trip

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

  stage_group<T, GLOBAL>(tb, G, L, rs, d, u, D, U, B, lds_raw, tid);

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
// Flow solve (ascending branches whose children hang off their far end, fast
// form, image in LDS).  One wave per group runs the group's static step
// schedule: at step t, lane l eliminates one compartment, stored at position
// R[t] + (active lanes below l), so the lanes of a step touch consecutive
// LDS entries.  Per position the image holds d, u, b (24 bytes); the
// backward sweep overwrites d with f = u / d' and b with y = b' / d', the
// forward sweep overwrites y with x.
//
// Contributions to a parent (paper §2: d_p -= u_i^2 / d'_i, b_p -= u_i b'_i / d'_i)
// travel in two ways.  Inside a branch, and from the heavy child into its
// parent (same lane, next step), the pair (f, b') stays in registers.  A
// light child adds its contribution to the parent's LDS entry (ds_add_f64)
// at its last step, at least two steps before the parent's first one.  The
// group is one wave and the LDS executes a wave's operations in order, so
// every read sees the additions issued in earlier steps.  The forward sweep
// replays the steps backwards: x of the parent is in registers (heavy child)
// or in LDS, written in an earlier forward step (light child).
// ---------------------------------------------------------------------------
using hines::flow_image8;
using hines::flow_lds_bytes;
using hines::flow_mask_offset;

__device__ __forceinline__ int tri(int p) { return (int)__umul24((unsigned)p, 3u); }  // 3 p, p < 2^24
__device__ __forceinline__ bool lane_in(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }
__device__ __forceinline__ int rank_in(uint64_t m, int base) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, (uint32_t)base));
}
typedef __attribute__((address_space(3))) double lds_f64;
typedef __attribute__((address_space(3))) int16_t lds_i16;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) u32x4 lds_u4;
typedef __attribute__((address_space(3))) uint8_t lds_u8;

__device__ __forceinline__ void lds_add(lds_f64* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Right-hand side forms of the flow kernel, fixed at compile time: given,
// c v, c v + i, c v + sigma Z.
enum : int { kFlowGiven = 0, kFlowCV = 1, kFlowCVI = 2, kFlowNoise = 3 };
// Cell-lane kernel only: eliminate the matrix alone and keep its factors.
enum : int { kCellFactor = 4 };
// kCellCond: the step of a model whose diagonal changes every step (a
// linearised membrane current g V - g E): the kernel assembles
// d_i = c_i + g_i + a_i + sum over children a_k from the edge conductances
// a = -u (paper §1) while it eliminates, with b = c v + g E.  The d argument
// carries g and rs.icur carries g E.
enum : int { kCellCond = 5 };

// Element e of a user range (user index lo + e) -> its position.  A lane
// handles elements lane, lane + 64, ...; the loads of kStageUnroll of them are
// issued before any is used.  Indices past the range are clamped to its last
// element, so every load is unconditional (the repeated element is written
// twice with the same value).
constexpr int kStageUnroll = 16;

// The first kStageUnroll entries of each lane are also returned in keep[], so
// that a group staged in one batch stores its solution without reading its
// positions again.
template <int RHS>
__device__ __forceinline__ void flow_stage_range(const RhsSpec& rs, const double* __restrict__ d_,
                                                 const double* __restrict__ u_, int64_t lo, int n,
                                                 const uint16_t* __restrict__ pos, lds_f64* img, int lane,
                                                 uint32_t* keep) {
  // uniform bases, 32-bit per-lane offsets
  const double* __restrict__ d = d_ + lo;
  const double* __restrict__ u = u_ + lo;
  const double* __restrict__ rhs = rs.rhs + lo;
  const double* __restrict__ cc = rs.c + lo;
  const double* __restrict__ vv = rs.v + lo;
  const double* __restrict__ ii = rs.icur + lo;
  for (int e0 = 0; e0 < n; e0 += 64 * kStageUnroll) {
    uint32_t pw[kStageUnroll];
    double dv[kStageUnroll], uv[kStageUnroll], bv[kStageUnroll], cv[kStageUnroll];
#pragma unroll
    for (int k = 0; k < kStageUnroll; ++k) {
      const int e = min(e0 + 64 * k + lane, n - 1);
      pw[k] = pos[e];
      dv[k] = d[e];
      uv[k] = u[e];
      if constexpr (RHS == kFlowGiven) {
        bv[k] = rhs[e];
      } else {
        cv[k] = cc[e];
        bv[k] = vv[e];
      }
    }
#pragma unroll
    for (int k = 0; k < kStageUnroll; ++k) {
      const int e = min(e0 + 64 * k + lane, n - 1);
      double b = bv[k];
      if constexpr (RHS != kFlowGiven) b = cv[k] * bv[k];
      if constexpr (RHS == kFlowCVI) b = b + ii[e];
      if constexpr (RHS == kFlowNoise) b = b + noise_draw(rs.seed, rs.step, (uint64_t)(lo + e), rs.sigma);
      lds_f64* q = img + (int)(pw[k] & 0x7fffu);
      q[0] = dv[k];
      q[1] = (pw[k] & 0x8000u) ? 0.0 : uv[k];
      q[2] = b;
    }
    if (e0 == 0) {
#pragma unroll
      for (int k = 0; k < kStageUnroll; ++k) keep[k] = pw[k];
    }
  }
}

// keep: the positions of the first batch (from the staging), or nullptr.
__device__ __forceinline__ void flow_store_range(double* x_, int64_t lo, int n, const uint16_t* __restrict__ pos,
                                                 const lds_f64* img, int lane, const uint32_t* keep) {
  double* x = x_ + lo;
  for (int e0 = 0; e0 < n; e0 += 64 * kStageUnroll) {
    uint32_t pw[kStageUnroll];
    if (e0 == 0 && keep) {
#pragma unroll
      for (int k = 0; k < kStageUnroll; ++k) pw[k] = keep[k];
    } else {
#pragma unroll
      for (int k = 0; k < kStageUnroll; ++k) pw[k] = pos[min(e0 + 64 * k + lane, n - 1)];
    }
#pragma unroll
    for (int k = 0; k < kStageUnroll; ++k) {
      const int e = e0 + 64 * k + lane;
      if (e < n) x[e] = img[(int)(pw[k] & 0x7fffu) + 2];
    }
  }
}

// Step masks: staged into LDS with the group (16 bytes per step: active and
// push masks); a step's masks are read one step ahead with a broadcast LDS
// read and moved to scalar registers.
__device__ __forceinline__ uint64_t first_u64(uint32_t lo, uint32_t hi) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)hi) << 32) |
         (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)lo);
}

// Both sweeps run the same straight-line code for every lane in every chunk
// step.  The chunk of a busy lane is one LDS block; sub-step j is entry j of
// the block, so every access of a sub-step is the block base plus an
// immediate offset.  An idle lane reads the identity block (d = 1, u = 0,
// b = 0 per entry, which eliminates to zeros) and writes into the sink, which
// is never read.  Only the pushes are masked.
constexpr int KC = hines::kFlowChunk;
constexpr int KB8 = hines::kFlowBlock8;

template <int RHS>
__global__ __launch_bounds__(64) void k_solve_flow(DevTables tb, RhsSpec rs, const double* __restrict__ d,
                                                   const double* __restrict__ u, double* x) {
  extern __shared__ __attribute__((aligned(16))) double img_raw[];
  lds_f64* img = (lds_f64*)img_raw;
  const int g = tb.glist[blockIdx.x];
  const KGroup G = tb.grp[g];
  const hines::KFlow W = tb.flow[g];
  const int lane = threadIdx.x;
  const uint16_t* pos = tb.fpos + W.pos_off;
  const int F = W.nstep;
  const int nblk = W.nent / KC;
  const int idle = nblk * KB8, sink = idle + KB8 + lane;
  lds_i16* aux = (lds_i16*)(img + flow_image8(W));
  // masks of steps 0 .. F-1, then one zero record on each side (steps -1 and F)
  lds_u4* msk = (lds_u4*)((lds_u8*)img + flow_mask_offset(W)) + 1;
  // masks and push targets by global->LDS DMA (16- and 4-byte units; the push
  // targets of a group start 4-byte aligned and the table is padded)
  dma16<64>(tb.fmask + 2 * W.step_off, (void*)(msk), F, lane);
  dma4<64>(tb.faux + W.aux_off, (void*)aux, (W.naux + 1) >> 1, lane);
  // every entry of every block (pads and the identity block included) starts
  // as the identity compartment; the scatter below overwrites the real ones
  for (int e = lane; e < W.nent + KC; e += 64) {
    const int o = (e / KC) * KB8 + 3 * (e % KC);
    img[o] = 1.0;
    img[o + 1] = 0.0;
    img[o + 2] = 0.0;
  }
  if (lane == 0) {
    msk[-1] = u32x4{0u, 0u, 0u, 0u};
    msk[F] = u32x4{0u, 0u, 0u, 0u};
    if (W.naux == 0) aux[0] = 0;  // the clamped push-target read stays defined
  }
  uint32_t keep[kStageUnroll];
  if (G.contig) {
    flow_stage_range<RHS>(rs, d, u, G.user_base + G.user_lo, G.user_n, pos, img, lane, keep);
  } else {
    int e0 = 0;
    for (int c = 0; c < G.ncell; ++c) {
      const KCell C = tb.cell[G.cell_begin + c];
      flow_stage_range<RHS>(rs, d, u, C.user_lo, C.n, pos + e0, img, lane, keep);
      e0 += C.n;
    }
  }
  __builtin_amdgcn_s_waitcnt(0);  // every DMA of this wave has landed
  __syncthreads();  // staged
  const int last_aux = W.naux > 0 ? W.naux - 1 : 0;

  // Backward sweep.  During chunk step t: the masks of t + 1 move to scalar
  // registers, the masks of t + 2, the operands of t + 1 and the push target of
  // t + 1 are read from LDS, and the KC sub-steps of t are eliminated.
  {
    const u32x4 m0 = msk[0];
    uint64_t M = first_u64(m0.x, m0.y), E = first_u64(m0.z, m0.w);
    u32x4 mv = msk[1];
    int R = 0, A = 0;
    int rb = lane_in(M) ? rank_in(M, 0) * KB8 : idle;
    double Dn[KC], Un[KC], Bn[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) {
      Dn[j] = img[rb + 3 * j];
      Un[j] = img[rb + 3 * j + 1];
      Bn[j] = img[rb + 3 * j + 2];
    }
    int qn = aux[min(rank_in(E, 0), last_aux)];
    double fin = 0.0, uin = 0.0, bin = 0.0;
    for (int t = 0; t < F; ++t) {
      const uint64_t M1 = first_u64(mv.x, mv.y), E1 = first_u64(mv.z, mv.w);
      mv = msk[t + 2 <= F ? t + 2 : F];
      const int R1 = R + __builtin_popcountll(M), A1 = A + __builtin_popcountll(E);
      double Dc[KC], Uc[KC], Bc[KC];
#pragma unroll
      for (int j = 0; j < KC; ++j) {
        Dc[j] = Dn[j];
        Uc[j] = Un[j];
        Bc[j] = Bn[j];
      }
      const int qp = qn;
      const int wb = lane_in(M) ? rb : sink;
      rb = lane_in(M1) ? rank_in(M1, R1) * KB8 : idle;
#pragma unroll
      for (int j = 0; j < KC; ++j) {
        Dn[j] = img[rb + 3 * j];
        Un[j] = img[rb + 3 * j + 1];
        Bn[j] = img[rb + 3 * j + 2];
      }
      qn = aux[min(rank_in(E1, A1), last_aux)];
#pragma unroll
      for (int j = 0; j < KC; ++j) {
        const double dl = __builtin_fma(-fin, uin, Dc[j]);
        const double bl = __builtin_fma(-fin, bin, Bc[j]);
        const double r = rcp_nr(dl);
        const double f = Uc[j] * r;
        img[wb + 3 * j] = f;
        img[wb + 3 * j + 2] = bl * r;
        fin = f;
        uin = Uc[j];
        bin = bl;
      }
      {
        const double cd = -(fin * uin), cb = -(fin * bin);
        if (lane_in(E)) {
          lds_add(img + qp, cd);
          lds_add(img + qp + 2, cb);
        }
      }
      fin = lane_in(M & ~E) ? fin : 0.0;
      M = M1;
      E = E1;
      R = R1;
      A = A1;
    }
  }
  __syncthreads();  // backward done

  // Forward sweep, chunk steps in reverse, sub-steps in reverse.  During step
  // t: the masks of t - 2 move to scalar registers, the masks of t - 3 are
  // read, the operands of t - 1, the parent x of the pushing lanes of t - 1 and
  // the push target of t - 2 are read from LDS, and step t is solved.
  {
    const u32x4 ma = msk[F - 1], mb = msk[F - 2];
    uint64_t M = first_u64(ma.x, ma.y), E = first_u64(ma.z, ma.w);
    uint64_t M1 = first_u64(mb.x, mb.y), E1 = first_u64(mb.z, mb.w);
    u32x4 mv = msk[F - 3 >= -1 ? F - 3 : -1];
    const int R = nblk - __builtin_popcountll(M), A = W.naux - __builtin_popcountll(E);
    int R1 = R - __builtin_popcountll(M1), A1 = A - __builtin_popcountll(E1);
    int rb = lane_in(M) ? rank_in(M, R) * KB8 : idle;
    double fn[KC], yn[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) {
      fn[j] = img[rb + 3 * j];
      yn[j] = img[rb + 3 * j + 2];
    }
    double xqn = img[aux[min(rank_in(E, A), last_aux)] + 2];
    int q1 = aux[min(rank_in(E1, A1), last_aux)];
    double xp = 0.0;
    for (int t = F - 1; t >= 0; --t) {
      const uint64_t M2 = first_u64(mv.x, mv.y), E2 = first_u64(mv.z, mv.w);
      mv = msk[t - 3 >= -1 ? t - 3 : -1];
      const int R2 = R1 - __builtin_popcountll(M2), A2 = A1 - __builtin_popcountll(E2);
      double fc[KC], yc[KC];
#pragma unroll
      for (int j = 0; j < KC; ++j) {
        fc[j] = fn[j];
        yc[j] = yn[j];
      }
      const double xq = xqn;
      const int wb = lane_in(M) ? rb : sink;
      rb = lane_in(M1) ? rank_in(M1, R1) * KB8 : idle;
#pragma unroll
      for (int j = 0; j < KC; ++j) {
        fn[j] = img[rb + 3 * j];
        yn[j] = img[rb + 3 * j + 2];
      }
      xqn = img[q1 + 2];
      q1 = aux[min(rank_in(E2, A2), last_aux)];
      double xv = lane_in(E) ? xq : xp;
#pragma unroll
      for (int j = KC - 1; j >= 0; --j) {
        xv = __builtin_fma(-fc[j], xv, yc[j]);
        img[wb + 3 * j + 2] = xv;
      }
      xp = lane_in(M) ? xv : xp;
      M = M1;
      E = E1;
      M1 = M2;
      E1 = E2;
      R1 = R2;
      A1 = A2;
    }
  }
  __syncthreads();  // forward done
  if (G.contig) {
    flow_store_range(x, G.user_base + G.user_lo, G.user_n, pos, img, lane, keep);
  } else {
    int e0 = 0;
    for (int c = 0; c < G.ncell; ++c) {
      const KCell C = tb.cell[G.cell_begin + c];
      flow_store_range(x, C.user_lo, C.n, pos + e0, img, lane, G.ncell == 1 ? keep : nullptr);
      e0 += C.n;
    }
  }
}

// ---------------------------------------------------------------------------
// Cell-lane solve: one lane per cell, 64 cells of similar size per wave.  Lane
// c walks its cell in the order of the setup tables (the reverse of a depth-
// first order in the backward sweep, that order in the forward sweep),
// kCellChunk steps per chunk.
//
// The inputs of a chunk are gathered by the whole wave: in slot r, lane j
// loads element j % K of the cell of lane (64 / K) r + j / K (K = kCellChunk,
// 16: lane 4 r + j / 16), so K lanes read one run of a cell's compartments.  They pass through two LDS planes (d, u and b;
// rows padded so that both the gathering writes and the per-lane reads are
// free of bank conflicts) to the lane that eliminates them.  The factors
// (f, y) of each step go to a device scratch in lane-major order (one 1 KiB
// store per step) and return in the forward sweep, whose x values pass back
// through LDS to the gather mapping for the store in user order.
//
// A long cell may be cut in two halves walked by lanes c < 32 (the subtree)
// and c + 32 (the rest); the cut edge's contribution and, in the forward
// sweep, the parent's x cross through mailbox slot c at strictly ordered steps.
//
// Contributions to a parent (paper §2: d_p -= u_i f_i, b_p -= u_i y_i) stay in
// registers when the parent is eliminated next.  The contributions of its
// other children wait in one merged stack entry per pending parent; the top
// entry lives in registers, the ones below in LDS slots (slot 0 is a dummy
// that lanes without an entry to spill write into).  The forward sweep keeps
// x of a compartment with several children on the same kind of stack.
// ---------------------------------------------------------------------------
constexpr int CK = hines::kCellChunk;
constexpr int CG = hines::kCellSlotCells;  // cells per gather slot (a run of CK lanes each)
// Rows padded by 256 / CK bytes: the gathering writes (CK lanes of one cell,
// consecutive elements, per phase of 16 or 32 lanes) and the per-lane reads
// then fall into distinct banks.
constexpr int kCellRowDU = 64 * 16 + 256 / CK;  // bytes per element row of the (d, u) plane
constexpr int kCellRowB = 64 * 8 + 256 / CK;    // bytes per element row of the b plane (x in the forward sweep)
constexpr int kCellLdsB = CK * kCellRowDU;                 // byte offset of the b plane
constexpr int kCellLdsStack = kCellLdsB + CK * kCellRowB;  // byte offset of the stack slots
constexpr int kCellLdsMail = kCellLdsStack + hines::kCellStack * 64 * 16;  // byte offset of the mailboxes
constexpr int kCellLds = kCellLdsMail + 64 * 16;
static_assert(CK == 8 || CK == 16, "chunk of 8 or 16 steps");

typedef double double2_t __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) double2_t lds_d2;
typedef __attribute__((address_space(3))) char lds_char;
// LDS double at an absolute byte address
__device__ __forceinline__ lds_f64* lds_at(int a) { return (lds_f64*)(uintptr_t)(unsigned)a; }
typedef unsigned int cflag_t __attribute__((ext_vector_type(CK / 4)));  // CK flag bytes of one lane

// The CK 16-bit positions of one lane's gather slots.
struct CellPos {
  u32x4 w[CK / 8];
};

__device__ __forceinline__ unsigned cell_byte(const cflag_t& v, int e) { return (v[e >> 2] >> (8 * (e & 3))) & 0xffu; }
// position of slot r; padding reads the cell's first compartment (its value is replaced later)
__device__ __forceinline__ unsigned cell_pos(const CellPos& p, int r) {
  return (p.w[r >> 3][(r & 7) >> 1] >> (16 * (r & 1))) & 0xffffu;
}

// Table and scratch traffic is read once per sweep: non-temporal, so that it
// does not push the gathered lines of d, u, b out of L2.
__device__ __forceinline__ CellPos pos_ld(const u32x4* p) {
  CellPos r;
#pragma unroll
  for (int i = 0; i < CK / 8; ++i) r.w[i] = __builtin_nontemporal_load(p + i);
  return r;
}
__device__ __forceinline__ cflag_t flag_ld(const cflag_t* p) { return __builtin_nontemporal_load(p); }

template <int RHS>
struct CellBatch {
  double dv[CK], uv[CK], bv[CK];
  double cv[(RHS == kFlowGiven || RHS == kCellFactor) ? 1 : CK];
  double iv[(RHS == kFlowCVI || RHS == kCellCond) ? CK : 1];
};

// MT: the storage type of the matrix (double, or float widened exactly)
template <int RHS, typename MT>
__device__ __forceinline__ void cell_load(CellBatch<RHS>& B, const RhsSpec& rs, const MT* __restrict__ d,
                                          const MT* __restrict__ u, const int64_t* base, const CellPos& P) {
#pragma unroll
  for (int r = 0; r < CK; ++r) {
    const unsigned p = cell_pos(P, r);
    const int64_t i = base[r] + (p == hines::kCellPadPos ? 0u : p);
    B.dv[r] = (double)d[i];
    B.uv[r] = (double)u[i];
    if constexpr (RHS == kCellFactor) {
      B.bv[r] = 0.0;
    } else if constexpr (RHS == kFlowGiven) {
      B.bv[r] = rs.rhs[i];
    } else {
      B.cv[r] = rs.c[i];
      B.bv[r] = rs.v[i];
      if constexpr (RHS == kFlowCVI || RHS == kCellCond) B.iv[r] = rs.icur[i];
    }
  }
}

// Into the LDS planes.  A padding element reads its cell's first compartment
// and a cell root has no coupling: both get u = 0, so they contribute nothing
// (d > 0 and b of the first compartment keep every value finite).
template <int RHS>
__device__ __forceinline__ void cell_put(const CellBatch<RHS>& B, const RhsSpec& rs, const int64_t* base,
                                         const CellPos& P, lds_char* lds, int lane) {
  const int e = lane % CK;
#pragma unroll
  for (int r = 0; r < CK; ++r) {
    const int c = CG * r + lane / CK;
    const unsigned p = cell_pos(P, r);
    double b = B.bv[r];
    if constexpr (RHS != kFlowGiven && RHS != kCellFactor) b = B.cv[r] * B.bv[r];
    if constexpr (RHS == kFlowCVI || RHS == kCellCond) b = b + B.iv[r];
    if constexpr (RHS == kFlowNoise)
      b = b + noise_draw(rs.seed, rs.step, (uint64_t)(base[r] + (p == hines::kCellPadPos ? 0u : p)), rs.sigma);
    const double uu = (p == 0u || p == hines::kCellPadPos) ? 0.0 : B.uv[r];
    double dd = B.dv[r];
    if constexpr (RHS == kCellCond) dd = (B.cv[r] + dd) - uu;  // c + g + a of the edge to the parent
    *(lds_d2*)(lds + e * kCellRowDU + c * 16) = double2_t{dd, uu};
    *(lds_f64*)(lds + kCellLdsB + e * kCellRowB + c * 8) = b;
  }
}

// Backward elimination of one chunk from the LDS planes; (f, y) per step into fy.
// mb: the mailboxes (slot c: the contribution of the cut-off subtree in lane c);
// msrc: the lane's source list, the next take in its low 6 bits.
// FACTOR: keep (f, 1 / d') instead of (f, y).  The contribution to the parent
// is (u f, f b'), the same products a solve with stored factors forms.
// COND: the parent's diagonal also takes the child's edge conductance a = -u,
// so the diagonal contribution is u f + u.
template <bool FACTOR = false, bool COND = false>
__device__ __forceinline__ void cell_backward(const cflag_t& f, const lds_d2* pdu, const lds_f64* pb, lds_d2* stk,
                                              lds_d2* mb, int lane, double& cd, double& cb, double& td, double& tb,
                                              int& m, double2_t* fy, unsigned& msrc) {
#pragma unroll
  for (int e = 0; e < CK; ++e) {
    const unsigned fe = cell_byte(f, e);
    const double2_t du = pdu[e * (kCellRowDU / 16)];
    double dd = du.x, bb = pb[e * (kCellRowB / 8)];
    const double uu = du.y;
    const double kc = (fe & hines::CF_TIP) ? 0.0 : 1.0;  // the carry enters unless this is a tip
    dd = __builtin_fma(-kc, cd, dd);
    bb = __builtin_fma(-kc, cb, bb);
    if (fe & hines::CF_MBIN) {  // a cut-off child's contribution, posted at an earlier step
      const double2_t mv = mb[msrc & 63u];
      msrc >>= 6;
      dd = dd - mv.x;
      bb = bb - mv.y;
    }
    if (fe & hines::CF_POP) {  // the merged entry of the other children; refill the top
      dd = dd - td;
      bb = bb - tb;
      m -= 1;
      const double2_t t = stk[64 * m];
      td = t.x;
      tb = t.y;
    }
    const double rr = rcp_nr(dd);
    const double fv = uu * rr, yv = bb * rr;
    cd = COND ? __builtin_fma(uu, fv, uu) : uu * fv;
    cb = fv * bb;
    if (fe & hines::CF_PUSH) {
      stk[64 * m] = double2_t{td, tb};
      m += 1;
      td = cd;
      tb = cb;
    }
    if (fe & hines::CF_MERGE) {
      td = td + cd;
      tb = tb + cb;
    }
    if (fe & hines::CF_MBOUT) mb[lane] = double2_t{cd, cb};
    fy[e] = double2_t{fv, FACTOR ? rr : yv};
  }
}

// Forward substitution of one chunk (steps in reverse); x per step into the
// b plane, then through the gather mapping to the user order.
__device__ __forceinline__ void cell_forward(const cflag_t& f, const CellPos& P, const double2_t* fy,
                                             lds_f64* pb, const lds_f64* xrd, lds_f64* stx, lds_d2* mb, int lane,
                                             double& xc, double& xt, int& m, double* x, const int64_t* base,
                                             unsigned& msrc) {
#pragma unroll
  for (int e = CK - 1; e >= 0; --e) {
    const unsigned fe = cell_byte(f, e);
    double xp = (fe & (hines::CF_PUSH | hines::CF_MERGE)) ? xt : xc;
    if (fe & hines::CF_MBOUT) xp = mb[lane].x;  // x of the parent, posted by the other half
    if (fe & hines::CF_PUSH) {
      m -= 1;
      xt = stx[64 * m];
    }
    // a padding step's factors were never stored: its value must not reach
    // the next step (a cell root multiplies it by f = 0)
    const double xv = (fe & hines::CF_PAD) ? 0.0 : __builtin_fma(-fy[e].x, xp, fy[e].y);
    if (fe & hines::CF_POP) {
      stx[64 * m] = xt;
      m += 1;
      xt = xv;
    }
    if (fe & hines::CF_MBIN) {
      mb[msrc & 63u].x = xv;
      msrc >>= 6;
    }
    xc = xv;
    pb[e * (kCellRowB / 8)] = xv;
  }
#pragma unroll
  for (int r = 0; r < CK; ++r) {
    const double xv = xrd[CG * r];
    const unsigned p = cell_pos(P, r);
    if (p != hines::kCellPadPos) x[base[r] + p] = xv;
  }
}

// The walk layout of the time loop with kept factors: per (wave chunk, pair q
// of steps 2q and 2q + 1, lane) one 16-byte unit, so a lane moves two steps
// with one load and a wave instruction covers 1 KiB.  Index in 16-byte units.
__device__ __forceinline__ int64_t walk_pair(int64_t chunk, int q, int lane) {
  return (chunk * (CK / 2) + q) * 64 + lane;
}

// f into F and 1 / d' into F + slots, both in the walk layout
__device__ __forceinline__ void factor_store(const double2_t* fy, double* F, int64_t slots, int64_t chunk, int lane) {
  double2_t* f2 = (double2_t*)F;
  double2_t* r2 = (double2_t*)(F + slots);
#pragma unroll
  for (int q = 0; q < CK / 2; ++q) {
    const int64_t o = walk_pair(chunk, q, lane);
    f2[o] = double2_t{fy[2 * q].x, fy[2 * q + 1].x};
    r2[o] = double2_t{fy[2 * q].y, fy[2 * q + 1].y};
  }
}

// MT = float: the matrix is stored in FP32 and widened exactly on load; the
// elimination and everything after it stay in FP64.
template <int RHS, typename MT = double>
__global__ __launch_bounds__(64) void k_solve_cells(DevTables tb, RhsSpec rs, const MT* __restrict__ d,
                                                    const MT* __restrict__ u, double* x) {
  __shared__ __attribute__((aligned(16))) char cl_raw[kCellLds];
  lds_char* lds = (lds_char*)cl_raw;
  const int lane = threadIdx.x;
  const hines::KCellWave W = tb.cwave[blockIdx.x];
  const int nk = W.nchunk;
  int64_t base[CK];
#pragma unroll
  for (int r = 0; r < CK; ++r) base[r] = tb.cbase[(int64_t)blockIdx.x * 64 + CG * r + lane / CK];
  constexpr int PS = 8 * CK;  // u32x4 words of positions per chunk
  const u32x4* posv = (const u32x4*)(tb.cpos + W.chunk_off * hines::kCellChunkElems) + (CK / 8) * lane;
  const cflag_t* flv = (const cflag_t*)(tb.cflag + W.chunk_off * hines::kCellChunkElems) + lane;  // + 64 per chunk
  double2_t* scr = (double2_t*)tb.cscr + W.chunk_off * (CK * 64) + lane;  // + CK * 64 per chunk
  lds_d2* stk = (lds_d2*)(lds + kCellLdsStack) + lane;                       // slot s at stk[64 s]
  lds_d2* mb = (lds_d2*)(lds + kCellLdsMail);
  const lds_d2* pdu = (const lds_d2*)lds + lane;
  lds_f64* pb = (lds_f64*)(lds + kCellLdsB) + lane;

  // ---- backward sweep: the gather of chunk k + 1 and the stores of chunk
  // k - 1 overlap the elimination of chunk k ----
  CellPos P = pos_ld(posv);
  cflag_t fl = flag_ld(flv);
  CellBatch<RHS> B;
  cell_load<RHS, MT>(B, rs, d, u, base, P);
  CellPos Q = pos_ld(posv + PS * min(1, nk - 1));
  double cd = 0.0, cb = 0.0, td = 0.0, tb_ = 0.0;
  int m = 0;
  double2_t fy[CK];
  const uint64_t ms = tb.cmsrc[(int64_t)blockIdx.x * 64 + lane];
  unsigned msb = (unsigned)ms, msf = (unsigned)(ms >> 32);
  cflag_t fprev = fl;
  for (int k = 0; k < nk; ++k) {
    cell_put<RHS>(B, rs, base, P, lds, lane);
    if (k > 0) {  // padding steps store nothing; the forward sweep reads their slots but
                  // uses no value of a padding step (no carry or stack leaves one)
      if constexpr (RHS == kCellFactor) {  // f and 1 / d' of every step at its walk slot
        factor_store(fy, x, tb.cslots, W.chunk_off + k - 1, lane);
      } else {
        double2_t* sk = scr + (k - 1) * (CK * 64);
#pragma unroll
        for (int e = 0; e < CK; ++e)
          if (!(cell_byte(fprev, e) & hines::CF_PAD)) __builtin_nontemporal_store(fy[e], sk + e * 64);
      }
    }
    const cflag_t f = fl;
    fprev = f;
    if (k + 1 < nk) {
      fl = flag_ld(flv + 64 * (k + 1));
      cell_load<RHS, MT>(B, rs, d, u, base, Q);
      P = Q;
      Q = pos_ld(posv + PS * min(k + 2, nk - 1));
    }
    cell_backward<RHS == kCellFactor, RHS == kCellCond>(f, pdu, pb, stk, mb, lane, cd, cb, td, tb_, m, fy, msb);
  }
  if constexpr (RHS == kCellFactor) {  // the last chunk's factors
    factor_store(fy, x, tb.cslots, W.chunk_off + nk - 1, lane);
    return;
  }
  // chunk nk - 1 stays in registers: it is the first one of the forward sweep.
  // The forward sweep reads back this wave's own scratch stores.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

  // ---- forward sweep: two register sets, the loads of the next chunk overlap
  // the substitution of this one ----
  lds_f64* stx = (lds_f64*)(lds + kCellLdsStack) + lane;  // slot s at stx[64 s]
  const lds_f64* xrd = (const lds_f64*)(lds + kCellLdsB + (lane % CK) * kCellRowB) + lane / CK;
  double xc = 0.0, xt = 0.0;
  m = 0;
  CellPos PA = pos_ld(posv + PS * (nk - 1)), PB = PA;
  cflag_t fa = flag_ld(flv + 64 * (nk - 1)), fb_ = fa;
  double2_t fb[CK];
  for (int k = nk - 1;; k -= 2) {
    if (k >= 1) {
      const double2_t* sk = scr + (k - 1) * (CK * 64);
#pragma unroll
      for (int e = 0; e < CK; ++e) fb[e] = __builtin_nontemporal_load(sk + e * 64);
      PB = pos_ld(posv + PS * (k - 1));
      fb_ = flag_ld(flv + 64 * (k - 1));
    }
    cell_forward(fa, PA, fy, pb, xrd, stx, mb, lane, xc, xt, m, x, base, msf);
    if (k < 1) break;
    if (k >= 2) {
      const double2_t* sk = scr + (k - 2) * (CK * 64);
#pragma unroll
      for (int e = 0; e < CK; ++e) fy[e] = __builtin_nontemporal_load(sk + e * 64);
      PA = pos_ld(posv + PS * (k - 2));
      fa = flag_ld(flv + 64 * (k - 2));
    }
    cell_forward(fb_, PB, fb, pb, xrd, stx, mb, lane, xc, xt, m, x, base, msf);
    if (k < 2) break;
  }
}

// ---------------------------------------------------------------------------
// Index-order cell lanes: the cell-lane solve with each lane walking its piece
// of a cell in decreasing user index (children before parents by the
// numbering of paper §2), kSeqChunk = 8 steps per chunk, so that a cell
// numbered level by level is gathered in long runs of whole lines.  The gather
// and the LDS planes are those of the cell-lane kernel at 8 steps (8 lanes read
// one 64-byte run of a lane's walk).  A contribution whose parent is not the
// next step is written or added into an LDS slot of the lane named by the
// step code, and the parent reads the slot; in the forward sweep the parent
// writes its x into that slot for the same children.  A cut-off subtree's root
// leaves through its lane's mailbox, as in the cell-lane kernel.
// ---------------------------------------------------------------------------
constexpr int SK = hines::kSeqChunk;
constexpr int SG = hines::kSeqSlotCells;
constexpr int kSeqRowDU = 64 * 16 + 256 / SK;  // the padding rule of the cell-lane planes
constexpr int kSeqRowB = 64 * 8 + 256 / SK;
constexpr int kSeqLdsB = SK * kSeqRowDU;
constexpr int kSeqLdsSlot = kSeqLdsB + SK * kSeqRowB;
constexpr int kSeqLdsMail = kSeqLdsSlot + hines::kSeqSlots * 64 * 16;
constexpr int kSeqLds = kSeqLdsMail + 64 * 16;
static_assert(SK == 8, "one 16-byte table word per lane and chunk");
static_assert(4 * kSeqLds <= 160 * 1024, "four waves per compute unit");

// 16-bit field r of a lane's 16-byte table word (positions or codes)
__device__ __forceinline__ unsigned seq_field(const u32x4& v, int r) { return (v[r >> 1] >> (16 * (r & 1))) & 0xffffu; }

// Register set of one backward chunk: the gathered d, u and right-hand side
// ingredients (b given; or c and v, with i for c v + i), and, for the noise
// form, the chunk's positions (the draw is keyed by the user index).
template <int RHS>
struct SeqSet {
  double d[SK], u[SK], b[SK];
  double c[RHS == kFlowGiven ? 1 : SK];
  double i[RHS == kFlowCVI ? SK : 1];
  u32x4 P;
};

template <int RHS>
__device__ __forceinline__ void seq_load(SeqSet<RHS>& S, const RhsSpec& rs, const double* __restrict__ d,
                                         const double* __restrict__ u, const int64_t* base, const u32x4& P) {
#pragma unroll
  for (int r = 0; r < SK; ++r) {
    const unsigned p = seq_field(P, r);
    const int64_t i = base[r] + (p == hines::kCellPadPos ? 0u : p);
    S.d[r] = d[i];
    S.u[r] = u[i];
    if constexpr (RHS == kFlowGiven) {
      S.b[r] = rs.rhs[i];
    } else {
      S.c[r] = rs.c[i];
      S.b[r] = rs.v[i];
      if constexpr (RHS == kFlowCVI) S.i[r] = rs.icur[i];
    }
  }
  if constexpr (RHS == kFlowNoise) S.P = P;
}

// Into the LDS planes, forming the right-hand side (the lane that eliminates
// an element zeroes its coupling when the step code marks padding or the
// cell root).
template <int RHS>
__device__ __forceinline__ void seq_put(const SeqSet<RHS>& S, const RhsSpec& rs, const int64_t* base,
                                        lds_char* lds, int lane) {
  const int e = lane % SK;
#pragma unroll
  for (int r = 0; r < SK; ++r) {
    const int c = SG * r + lane / SK;
    double bb = S.b[r];
    if constexpr (RHS != kFlowGiven) bb = S.c[r] * S.b[r];
    if constexpr (RHS == kFlowCVI) bb = bb + S.i[r];
    if constexpr (RHS == kFlowNoise) {
      const unsigned p = seq_field(S.P, r);
      bb = bb + noise_draw(rs.seed, rs.step, (uint64_t)(base[r] + (p == hines::kCellPadPos ? 0u : p)), rs.sigma);
    }
    *(lds_d2*)(lds + e * kSeqRowDU + c * 16) = double2_t{S.d[r], S.u[r]};
    *(lds_f64*)(lds + kSeqLdsB + e * kSeqRowB + c * 8) = bb;
  }
}

// Backward elimination of one chunk; (f, y) per step into fy.  slot: the
// lane's slot 1 at slot[0], slot s at slot[64 (s - 1)].
__device__ __forceinline__ void seq_backward(const u32x4& cw, const lds_d2* pdu, const lds_f64* pb, lds_d2* slot,
                                             lds_d2* mb, int lane, double& cd, double& cb, double2_t* fy,
                                             unsigned& msrc) {
#pragma unroll
  for (int e = 0; e < SK; ++e) {
    const unsigned q = seq_field(cw, e);
    const double2_t du = pdu[e * (kSeqRowDU / 16)];
    double dd = du.x, bb = pb[e * (kSeqRowB / 8)];
    // padding (d and b of the cell's first compartment) and the cell root have no coupling
    const double uu = (q & (hines::SQ_PAD | hines::SQ_ROOT)) ? 0.0 : du.y;
    const double kc = (q & hines::SQ_TIP) ? 0.0 : 1.0;  // the previous step is this one's child
    dd = __builtin_fma(-kc, cd, dd);
    bb = __builtin_fma(-kc, cb, bb);
    if (q & hines::SQ_MBIN) {  // a cut-off subtree's contribution, posted at an earlier step
      const double2_t mv = mb[msrc & 63u];
      msrc >>= 6;
      dd = dd - mv.x;
      bb = bb - mv.y;
    }
    const unsigned rs = (q >> hines::SQ_READ_SHIFT) & hines::SQ_SLOT;
    if (rs) {  // the other children's contributions
      const double2_t t = slot[64 * (rs - 1)];
      dd = dd - t.x;
      bb = bb - t.y;
    }
    const double rr = rcp_nr(dd);
    const double fv = uu * rr, yv = bb * rr;
    cd = uu * fv;
    cb = fv * bb;
    const unsigned ds = q & hines::SQ_SLOT;
    if (ds) {
      lds_d2* sp = slot + 64 * (ds - 1);
      *sp = (q & hines::SQ_FIRST) ? double2_t{cd, cb} : *sp + double2_t{cd, cb};
    }
    if (q & hines::SQ_MBOUT) mb[lane] = double2_t{cd, cb};
    fy[e] = double2_t{fv, yv};
  }
}

// Forward substitution of one chunk (steps in reverse), then the stores in
// the user order through the gather mapping.
__device__ __forceinline__ void seq_forward(const u32x4& cw, const u32x4& P, const double2_t* fy, lds_f64* pb,
                                            const lds_f64* xrd, lds_d2* slot, lds_d2* mb, int lane, double& xc,
                                            double* x, const int64_t* base, unsigned& msrc) {
#pragma unroll
  for (int e = SK - 1; e >= 0; --e) {
    const unsigned q = seq_field(cw, e);
    double xp = xc;  // the parent is the step after this one, unless named below
    const unsigned ds = q & hines::SQ_SLOT;
    if (ds) xp = ((lds_f64*)(slot + 64 * (ds - 1)))[0];
    if (q & hines::SQ_MBOUT) xp = mb[lane].x;
    // a padding step's factors are not used: its value must not reach a later step
    const double xv = (q & hines::SQ_PAD) ? 0.0 : __builtin_fma(-fy[e].x, xp, fy[e].y);
    const unsigned rs = (q >> hines::SQ_READ_SHIFT) & hines::SQ_SLOT;
    if (rs) ((lds_f64*)(slot + 64 * (rs - 1)))[0] = xv;
    if (q & hines::SQ_MBIN) {
      mb[msrc & 63u].x = xv;
      msrc >>= 6;
    }
    xc = xv;
    pb[e * (kSeqRowB / 8)] = xv;
  }
  // (a padding element stores nothing: redirecting its 8 bytes elsewhere
  // costs partial-line writes, measured slower than the branch)
#pragma unroll
  for (int r = 0; r < SK; ++r) {
    const double xv = xrd[SG * r];
    const unsigned p = seq_field(P, r);
    if (p != hines::kCellPadPos) x[base[r] + p] = xv;
  }
}

// Register set of one forward chunk: its factors, positions and codes.
struct SeqFwd {
  double2_t fy[SK];
  u32x4 P, c;
};

template <int RHS>
__global__ __launch_bounds__(64) void k_solve_seq(DevTables tb, RhsSpec rs, const double* __restrict__ d,
                                                  const double* __restrict__ u, double* x) {
  __shared__ __attribute__((aligned(16))) char sq_raw[kSeqLds];
  lds_char* lds = (lds_char*)sq_raw;
  const int lane = threadIdx.x;
  const hines::KCellWave W = tb.swave[blockIdx.x];
  const int nk = W.nchunk;
  int64_t base[SK];
#pragma unroll
  for (int r = 0; r < SK; ++r) base[r] = tb.sbase[(int64_t)blockIdx.x * 64 + SG * r + lane / SK];
  const u32x4* posv = (const u32x4*)(tb.spos + W.chunk_off * hines::kSeqChunkElems) + lane;   // + 64 per chunk
  const u32x4* codv = (const u32x4*)(tb.scode + W.chunk_off * hines::kSeqChunkElems) + lane;  // + 64 per chunk
  double2_t* scr = (double2_t*)tb.cscr + W.chunk_off * (SK * 64) + lane;                      // + SK * 64 per chunk
  lds_d2* slot = (lds_d2*)(lds + kSeqLdsSlot) + lane;
  lds_d2* mb = (lds_d2*)(lds + kSeqLdsMail);
  const lds_d2* pdu = (const lds_d2*)lds + lane;
  lds_f64* pb = (lds_f64*)(lds + kSeqLdsB) + lane;
  auto chunk = [&](int k) { return 64 * max(0, min(k, nk - 1)); };  // table offset of chunk k, clamped

  // ---- backward sweep.  Memory latency under load is microseconds while a
  // chunk's elimination takes a few hundred cycles, so the gathers run two
  // chunks ahead (two register sets, used in turn), the positions four and
  // the codes two.  Every load is unconditional (clamped to the last chunk):
  // the loop body stays straight-line and each wait covers only the data it
  // needs.  Loads land in the registers that use them: no copies. ----
  // (the prologue issues in the steady state's order: each position load
  // right after the gathers that used its registers)
  SeqSet<RHS> SA, SB;
  u32x4 PA = __builtin_nontemporal_load(posv), PB = __builtin_nontemporal_load(posv + chunk(1));
  u32x4 cA = __builtin_nontemporal_load(codv), cB = __builtin_nontemporal_load(codv + chunk(1));
  seq_load(SA, rs, d, u, base, PA);
  PA = __builtin_nontemporal_load(posv + chunk(2));
  seq_load(SB, rs, d, u, base, PB);
  PB = __builtin_nontemporal_load(posv + chunk(3));
  double cd = 0.0, cb = 0.0;
  double2_t fy[SK];
  const uint64_t ms = tb.smsrc[(int64_t)blockIdx.x * 64 + lane];
  unsigned msb = (unsigned)ms, msf = (unsigned)(ms >> 32);
  auto bstep = [&](int k, SeqSet<RHS>& S, u32x4& Pn, u32x4& cc) {
    seq_put(S, rs, base, lds, lane);                      // chunk k
    seq_load(S, rs, d, u, base, Pn);                      // chunk k + 2
    Pn = __builtin_nontemporal_load(posv + chunk(k + 4));
    seq_backward(cc, pdu, pb, slot, mb, lane, cd, cb, fy, msb);
    // every step stored, padding too (into its own entry, never used): whole
    // 1 KiB rows, and no branch splits the bookkeeping of outstanding memory
    // operations (skipping padding measured slower)
    double2_t* sk = scr + (int64_t)k * (SK * 64);
#pragma unroll
    for (int e = 0; e < SK; ++e) __builtin_nontemporal_store(fy[e], sk + e * 64);
    cc = __builtin_nontemporal_load(codv + chunk(k + 2));
  };
  for (int k = 0;; k += 2) {
    bstep(k, SA, PA, cA);
    if (k + 1 >= nk) break;
    bstep(k + 1, SB, PB, cB);
    if (k + 2 >= nk) break;
  }
  // the forward sweep reads back this wave's own scratch stores
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

  // ---- forward sweep: chunks nk - 1 down to 0, three register sets in turn,
  // so that the loads of the next three chunks are in flight while one is
  // substituted.  Chunk nk - 1's factors are still in fy. ----
  const lds_f64* xrd = (const lds_f64*)(lds + kSeqLdsB + (lane % SK) * kSeqRowB) + lane / SK;
  double xc = 0.0;
  SeqFwd FA, FB, FC;
  auto fload = [&](SeqFwd& F, int k) {
    const int kc = max(k, 0);
    const double2_t* sk = scr + (int64_t)kc * (SK * 64);
#pragma unroll
    for (int e = 0; e < SK; ++e) F.fy[e] = __builtin_nontemporal_load(sk + e * 64);
    F.P = __builtin_nontemporal_load(posv + chunk(kc));
    F.c = __builtin_nontemporal_load(codv + chunk(kc));
  };
#pragma unroll
  for (int e = 0; e < SK; ++e) FA.fy[e] = fy[e];
  FA.P = __builtin_nontemporal_load(posv + chunk(nk - 1));
  FA.c = __builtin_nontemporal_load(codv + chunk(nk - 1));
  fload(FB, nk - 2);
  fload(FC, nk - 3);
  auto fstep = [&](int k, SeqFwd& F) {
    seq_forward(F.c, F.P, F.fy, pb, xrd, slot, mb, lane, xc, x, base, msf);
    fload(F, k - 3);
  };
  for (int k = nk - 1;; k -= 3) {
    fstep(k, FA);
    if (k < 1) break;
    fstep(k - 1, FB);
    if (k < 2) break;
    fstep(k - 2, FC);
    if (k < 3) break;
  }
}

// ---------------------------------------------------------------------------
// LDS-resident solve: one wave per group of whole cells.  The group's d, u, b
// are staged into LDS once by global->LDS DMA, as three planes of S slots in
// the user numbering (slot s = user index lo + s); the sweeps touch only LDS;
// the solution leaves in coalesced 16-byte stores.
//
// Backward sweep (paper §2: every compartment after its children).  Each lane
// runs its path records in chunk order, kResK steps per chunk: a path is
// eliminated from its bottom (a leaf, after any padding steps on the zero
// entry) to its top in consecutive steps, so the contribution (u f, u y) to
// the next compartment stays in registers; at the end of its last chunk it is
// added into the parent's LDS entry (d_p -= u f, b_p -= u y) unless the top is
// a cell root.  A lane reads the operands of its next active chunk while the
// current one runs; setup ends every light path two chunks before the chunk
// that eliminates its parent, so each compartment is read after all its
// children have contributed (the wave executes its LDS operations in order).
// A step stores f = u / d' over u and y = b' / d' over b.
//
// Forward sweep: the chunks in reverse.  A path runs from its top (x of the
// parent read from LDS, written at least two chunks earlier; zero for a root)
// down to its bottom: x_j = y_j - f_j x_parent, written over y.  Lanes with no
// path in a chunk are masked off for the whole chunk.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) uint16_t lds_u16;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) u32x2 lds_u2;

struct ResRec {
  int c0, cend, par;
};
// a record word as loaded; decoded only where it is used, so the LDS read of a
// lane's next record is not waited for at once.  Every lane's records are
// enclosed by idle sentinels (first chunk 65535, no chunks): reading one
// record past either end needs no bounds test.
__device__ __forceinline__ ResRec res_decode(u32x2 w) {
  ResRec r;
  r.c0 = (int)(w.x & 0xffffu);
  r.cend = r.c0 + (int)(w.x >> 16);
  r.par = (int)(w.y & 0xffffu);
  return r;
}
// keep the decoded fields computed here (not sunk past a later load of the word)
__device__ __forceinline__ void res_pin(ResRec& r) { __asm__ volatile("" : "+v"(r.c0), "+v"(r.cend), "+v"(r.par)); }

// s_waitcnt lgkmcnt(0) with the vector-memory and export counters left free
constexpr int kWaitLgkm0 = 0xc07f;

// slot-list entry: the byte offsets (uint16) of a chunk's kResK steps
template <int KK>
struct ResEntOf;
template <>
struct ResEntOf<4> {
  typedef u32x2 type;
};
template <>
struct ResEntOf<8> {
  typedef u32x4 type;
};
typedef ResEntOf<hines::kResK>::type res_ent;
typedef __attribute__((address_space(3))) res_ent lds_ent;
static_assert(sizeof(res_ent) == hines::kResEntBytes, "slot-list entry");

__device__ __forceinline__ int res_a(res_ent a, int k) {
  const unsigned w = a[k >> 1];
  return (int)((k & 1) ? (w >> 16) : (w & 0xffffu));
}

// (d, u) of a step in one register pair: the two plane reads merge into one
// ds_read2st64 whose destination is the pair
template <int S>
__device__ __forceinline__ void res_load_bwd(const lds_char* base, const int (&o4)[hines::kResK],
                                             double2_t (&odu)[hines::kResK], double (&ob)[hines::kResK]) {
#pragma unroll
  for (int k = 0; k < hines::kResK; ++k) {
    const int o = o4[k];
    double2_t v;
    v.x = *lds_at(o);
    v.y = *lds_at(8 * S + o);
    odu[k] = v;
    ob[k] = *lds_at(16 * S + o);
  }
}

// (f, y) of a step
template <int S>
__device__ __forceinline__ void res_load_fwd(const lds_char* base, const int (&o4)[hines::kResK],
                                             double2_t (&ofy)[hines::kResK]) {
#pragma unroll
  for (int k = 0; k < hines::kResK; ++k) {
    const int o = o4[k];
    double2_t v;
    v.x = *lds_at(8 * S + o);
    v.y = *lds_at(16 * S + o);
    ofy[k] = v;
  }
}

// one backward chunk: eliminate kResK steps, then store f and y (each value in
// a register of its own, so no store holds up the next step's arithmetic)
template <int S>
__device__ __forceinline__ void res_elim(lds_char* base, const int (&o4)[hines::kResK], const double2_t (&odu)[hines::kResK],
                                         const double (&ob)[hines::kResK], double& ncd, double& ncb) {
  double fv[hines::kResK], yv[hines::kResK];
#pragma unroll
  for (int k = 0; k < hines::kResK; ++k) {
    const double uk = odu[k].y;
    const double dd = odu[k].x + ncd;
    const double bb = ob[k] + ncb;
    const double r = rcp_nr(dd);
    fv[k] = uk * r;
    yv[k] = bb * r;
    // u^2 / d' with u^2 formed off the chain of dependent steps (u is read a
    // chunk ahead): the next pivot waits on one product less
    ncd = -((uk * uk) * r);
    ncb = -(uk * yv[k]);
  }
#pragma unroll
  for (int k = 0; k < hines::kResK; ++k) {
    *lds_at(8 * S + o4[k]) = fv[k];
    *lds_at(16 * S + o4[k]) = yv[k];
  }
}

template <int S>
__device__ __forceinline__ void res_subst(lds_char* base, const int (&o4)[hines::kResK], const double2_t (&ofy)[hines::kResK],
                                          double& xp) {
  double xv[hines::kResK];
#pragma unroll
  for (int k = hines::kResK - 1; k >= 0; --k) {
    xv[k] = __builtin_fma(-ofy[k].x, xp, ofy[k].y);
    xp = xv[k];
  }
#pragma unroll
  for (int k = hines::kResK - 1; k >= 0; --k) *lds_at(16 * S + o4[k]) = xv[k];
}

template <int S>
__global__ __launch_bounds__(64) void k_solve_res(DevTables tb, const double* __restrict__ d,
                                                  const double* __restrict__ u, const double* __restrict__ b,
                                                  double* __restrict__ x) {
  constexpr int K = hines::kResK;
  extern __shared__ __attribute__((aligned(16))) double res_raw[];
  const hines::KResGroup G = tb.rgrp[tb.rlist[blockIdx.x]];
  const int lane = threadIdx.x;
  // the group's image starts at LDS address 0 (the kernel declares no other
  // LDS): list entries and record fields are absolute LDS byte addresses
  lds_char* base = (lds_char*)res_raw;
  constexpr int oU = 8 * S, oB = 16 * S, oBlob = 24 * S;
  lds_f64* D = (lds_f64*)base;
  lds_f64* U = (lds_f64*)(base + oU);
  lds_f64* B = (lds_f64*)(base + oB);
  // ---- staging ----
  const int nu = G.ndma >> 1;
  char* gbase = (char*)res_raw;  // generic pointer for the DMA helper
  dma16<64>(d + G.lo, gbase, nu, lane);
  dma16<64>(u + G.lo, gbase + oU, nu, lane);
  dma16<64>(b + G.lo, gbase + oB, nu, lane);
  dma16<64>(tb.rblob + 16 * G.blob, gbase + oBlob, G.blob_units, lane);
  double tail_d = 0.0, tail_u = 0.0, tail_b = 0.0;
  const bool tail = (G.ndma & 1) && lane == 0;
  if (tail) {
    tail_d = d[G.lo + G.ndma - 1];
    tail_u = u[G.lo + G.ndma - 1];
    tail_b = b[G.lo + G.ndma - 1];
  }
  __builtin_amdgcn_s_waitcnt(0);  // every DMA of this wave has landed
  const int zero = G.nslot;
  if (tail) {
    D[G.ndma - 1] = tail_d;
    U[G.ndma - 1] = tail_u;
    B[G.ndma - 1] = tail_b;
  }
  if (lane == 0) {  // the zero entry: eliminates to nothing
    D[zero] = 1.0;
    U[zero] = 0.0;
    B[zero] = 0.0;
  }
  const lds_u16* ltab = (const lds_u16*)(base + oBlob);
  const lds_u16* roots = ltab + hines::kResLaneTab / 2;
  // cells re-rooted at their centre: on the path from the old root to the new
  // one every compartment takes as coupling to its new parent the u staged at
  // that parent (its old child); a batch reads all its sources before it
  // writes, and a later batch reads no slot an earlier one wrote
  const lds_u16* flips = roots + ((2 * G.nroot + 15) & ~15) / 2;
  for (int q0 = 0; q0 < G.nflip; q0 += 64) {
    const int q = q0 + lane;
    int dst = zero;
    double v = 0.0;
    if (q < G.nflip) {
      dst = flips[2 * q];
      v = U[flips[2 * q + 1]];
    }
    __asm__ volatile("" ::: "memory");
    if (q < G.nflip) U[dst] = v;
    __asm__ volatile("" ::: "memory");
  }
  for (int r = lane; r < G.nroot; r += 64) U[roots[r]] = 0.0;  // a root has no coupling
  const lds_u2* recs = (const lds_u2*)(base + oBlob + G.rec_off);
  const lds_ent* lists = (const lds_ent*)(base + oBlob + G.list_off);
  const int kb = ltab[lane], ke = ltab[lane + 1] - 1;  // records [kb, ke), sentinels at kb - 1 and ke
  const int lb = ltab[65 + lane], le = ltab[65 + lane + 1];
  const int NC = G.nchunk;
  __asm__ volatile("" ::: "memory");

  // ---- backward sweep ----
  {
    int ri = kb;
    ResRec R = res_decode(recs[ri]);
    u32x2 Rn = recs[ri + 1];  // the next record, raw
    res_ent ahead = lists[lb];  // the list region holds one spare entry past the last
    int li = lb + 1;
    double2_t du0[K] = {}, du1[K] = {};
    double b0[K] = {}, b1[K] = {};
    int a0[K] = {}, a1[K] = {};  // byte offsets of the chunk's steps
    double ncd = 0.0, ncb = 0.0;
    // operands of chunk c1 for the lanes active in it (the next list entry)
    auto pre = [&](int c1, int (&anx)[K], double2_t (&dun)[K], double (&bn)[K]) {
      const bool act1 = c1 < R.cend ? c1 >= R.c0 : c1 >= (int)(Rn.x & 0xffffu);
      if (act1 && c1 < NC) {
#pragma unroll
        for (int k = 0; k < K; ++k) anx[k] = res_a(ahead, k);
        res_load_bwd<S>(base, anx, dun, bn);
        __builtin_amdgcn_sched_barrier(0);
        ahead = lists[li];
        li += 1;
      }
    };
    // one chunk: prefetch the next chunk's operands, eliminate, push
    auto chunk = [&](int c, int (&acur)[K], double2_t (&duc)[K], double (&bc)[K], int (&anx)[K], double2_t (&dun)[K],
                     double (&bn)[K]) {
      // the operands of chunk c (read during the chunk before) have landed;
      // waiting here, where every lane passes, spares the masked blocks below
      // a wait of their own
      __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
      pre(c + 1, anx, dun, bn);
      __asm__ volatile("" ::: "memory");
      if (c >= R.c0 && c < R.cend) {
        res_elim<S>(base, acur, duc, bc, ncd, ncb);
        if (c == R.cend - 1) {  // the path's top
          if (R.par != hines::kResNoParent) {
            lds_add(lds_at(R.par), ncd);
            lds_add(lds_at(oB + R.par), ncb);
          }
          ncd = 0.0;
          ncb = 0.0;
          ri += 1;
          R = res_decode(Rn);
          res_pin(R);
          Rn = recs[ri + 1];
        }
      }
      __asm__ volatile("" ::: "memory");
    };
    pre(0, a0, du0, b0);
    for (int c = 0; c < NC; c += 2) {
      chunk(c, a0, du0, b0, a1, du1, b1);
      if (c + 1 < NC) chunk(c + 1, a1, du1, b1, a0, du0, b0);
    }
  }
  __asm__ volatile("" ::: "memory");

  // ---- forward sweep: chunks in reverse, records in reverse ----
  {
    int ri = ke - 1;
    ResRec R = res_decode(recs[ri]);
    u32x2 Rp = recs[ri - 1];  // the previous record, raw
    res_ent ahead = lists[le > lb ? le - 1 : lb];
    int li = le - 2;
    double2_t fy0[K] = {}, fy1[K] = {};
    double xq0 = 0.0, xq1 = 0.0;  // x of the parent of a top chunk's top
    int a0[K] = {}, a1[K] = {};
    double xp = 0.0;
    // operands of chunk c1 (and x of its top's parent) for the lanes active in it
    auto pre = [&](int c1, int (&anx)[K], double2_t (&fyn)[K], double& xqn) {
      const bool inR = c1 >= R.c0;
      const ResRec Q = inR ? R : res_decode(Rp);
      if (c1 >= Q.c0 && c1 < Q.cend && c1 >= 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) anx[k] = res_a(ahead, k);
        res_load_fwd<S>(base, anx, fyn);
        const int pq = Q.par != hines::kResNoParent && c1 == Q.cend - 1 ? Q.par : 8 * zero;
        xqn = *lds_at(oB + pq);
        __builtin_amdgcn_sched_barrier(0);
        ahead = lists[li < lb ? lb : li];
        li -= 1;
      }
    };
    auto chunk = [&](int c, int (&acur)[K], double2_t (&fyc)[K], double& xqc, int (&anx)[K], double2_t (&fyn)[K],
                     double& xqn) {
      __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
      pre(c - 1, anx, fyn, xqn);
      __asm__ volatile("" ::: "memory");
      if (c >= R.c0 && c < R.cend) {
        if (c == R.cend - 1) xp = xqc;
        res_subst<S>(base, acur, fyc, xp);
        if (c == R.c0) {  // the path's bottom: previous record
          ri -= 1;
          R = res_decode(Rp);
          res_pin(R);
          Rp = recs[ri - 1];
        }
      }
      __asm__ volatile("" ::: "memory");
    };
    pre(NC - 1, a0, fy0, xq0);
    for (int c = NC - 1; c >= 0; c -= 2) {
      chunk(c, a0, fy0, xq0, a1, fy1, xq1);
      if (c - 1 >= 0) chunk(c - 1, a1, fy1, xq1, a0, fy0, xq0);
    }
  }
  __asm__ volatile("" ::: "memory");

  // ---- store slots [first, first + count) ----
  const int s0 = G.first, s1 = G.first + G.count;
  double* xo = x + G.lo;
  for (int k = lane; 2 * k < s1; k += 64) {
    const int a = 2 * k;
    if (a >= s0 && a + 1 < s1) {
      *(double2_t*)(xo + a) = *(const lds_d2*)(B + a);
    } else {
      if (a >= s0 && a < s1) xo[a] = B[a];
      if (a + 1 >= s0 && a + 1 < s1) xo[a + 1] = B[a + 1];
    }
  }
}
// ---------------------------------------------------------------------------
// Time loop with the factors kept (cell-lane plans).  The matrix of a time
// loop does not change between steps, so the elimination of A (paper §2: the
// pivots d' and f = u / d') is done once per loop launch and each step only
// sweeps the right-hand side: y = (b - sum f_c b'_c) / d' backwards, x = y -
// f x_p forwards.  Everything a step touches (f, 1 / d', c, the current, V)
// lives in the walk layout (walk_pair): a lane moves two steps per 16-byte
// access and each wave instruction is one coalesced KiB.  V enters the walk
// layout at the start of a launch and returns to the user layout at its end.
// ---------------------------------------------------------------------------
struct CellLoop {
  const double* f;   // f = u / d' per walk slot
  const double* r;   // 1 / d'
  const double* c;   // c
  const double* ci;  // kFlowCVI: the current I
  double* v;         // V, then y and x in place
  const uint16_t* lp;  // kFlowNoise: positions, CK per lane and chunk (the user index of the draw)
  double sigma;
  uint32_t seed, step;
};

// user layout -> walk layout (padding slots get the cell's first compartment)
__global__ __launch_bounds__(64) void k_cells_to_walk(DevTables tb, const double* __restrict__ src,
                                                      double* __restrict__ dst) {
  __shared__ __attribute__((aligned(16))) char raw[CK * kCellRowB];
  lds_f64* pl = (lds_f64*)raw;
  const int lane = threadIdx.x;
  const hines::KCellWave W = tb.cwave[blockIdx.x];
  int64_t base[CK];
#pragma unroll
  for (int r = 0; r < CK; ++r) base[r] = tb.cbase[(int64_t)blockIdx.x * 64 + CG * r + lane / CK];
  constexpr int PS = 8 * CK;
  const u32x4* posv = (const u32x4*)(tb.cpos + W.chunk_off * hines::kCellChunkElems) + (CK / 8) * lane;
  const int wo = (lane % CK) * (kCellRowB / 8) + lane / CK;  // + CG r
  double2_t* d2 = (double2_t*)dst;
  for (int k = 0; k < W.nchunk; ++k) {
    const CellPos P = pos_ld(posv + PS * k);
    double v[CK];
#pragma unroll
    for (int r = 0; r < CK; ++r) {
      const unsigned p = cell_pos(P, r);
      v[r] = src[base[r] + (p == hines::kCellPadPos ? 0u : p)];
    }
#pragma unroll
    for (int r = 0; r < CK; ++r) pl[wo + CG * r] = v[r];
#pragma unroll
    for (int q = 0; q < CK / 2; ++q)
      d2[walk_pair(W.chunk_off + k, q, lane)] =
          double2_t{pl[2 * q * (kCellRowB / 8) + lane], pl[(2 * q + 1) * (kCellRowB / 8) + lane]};
  }
}

// walk layout -> user layout (padding slots are not stored)
__global__ __launch_bounds__(64) void k_cells_from_walk(DevTables tb, const double* __restrict__ src,
                                                        double* __restrict__ dst) {
  __shared__ __attribute__((aligned(16))) char raw[CK * kCellRowB];
  lds_f64* pl = (lds_f64*)raw;
  const int lane = threadIdx.x;
  const hines::KCellWave W = tb.cwave[blockIdx.x];
  int64_t base[CK];
#pragma unroll
  for (int r = 0; r < CK; ++r) base[r] = tb.cbase[(int64_t)blockIdx.x * 64 + CG * r + lane / CK];
  constexpr int PS = 8 * CK;
  const u32x4* posv = (const u32x4*)(tb.cpos + W.chunk_off * hines::kCellChunkElems) + (CK / 8) * lane;
  const lds_f64* rd = (const lds_f64*)((lds_char*)raw + (lane % CK) * kCellRowB) + lane / CK;
  const double2_t* s2 = (const double2_t*)src;
  for (int k = 0; k < W.nchunk; ++k) {
    const CellPos P = pos_ld(posv + PS * k);
#pragma unroll
    for (int q = 0; q < CK / 2; ++q) {
      const double2_t v = s2[walk_pair(W.chunk_off + k, q, lane)];
      pl[2 * q * (kCellRowB / 8) + lane] = v.x;
      pl[(2 * q + 1) * (kCellRowB / 8) + lane] = v.y;
    }
#pragma unroll
    for (int r = 0; r < CK; ++r) {
      const unsigned p = cell_pos(P, r);
      const double v = rd[CG * r];
      if (p != hines::kCellPadPos) dst[base[r] + p] = v;
    }
  }
}

// positions in lane order, CK per lane and chunk like the flags (for the draws)
__global__ void k_cells_lane_pos(DevTables tb, uint16_t* __restrict__ lp, int64_t nchunks) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nchunks * 64 * CK) return;
  const int64_t g = t / (64 * CK);
  const int c = (int)((t / CK) % 64), e = (int)(t % CK);
  lp[t] = tb.cpos[hines::cell_pos_index(g, c, e)];
}

// One implicit-Euler step with the factors kept: V <- A^-1 (c V + I) in the
// walk layout.  Two register sets: the loads of the next chunk are in flight
// while this one is swept.
__device__ __forceinline__ double pair_at(const double2_t* a, int e) { return (e & 1) ? a[e >> 1].y : a[e >> 1].x; }

template <int RHS>
struct StepChunk {
  double2_t f[CK / 2], r[CK / 2], c[CK / 2], i[RHS == kFlowCVI ? CK / 2 : 1], v[CK / 2];
  cflag_t fl;
  CellPos p;  // kFlowNoise: positions of the lane's steps
};

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt not waited for).  Issued once after
// the per-lane lists are loaded at the step kernel's start: the loop then
// updates them with plain ALU operations, and the compiler no longer counts
// them as loads that may still be in flight (which made it wait for every
// load in flight, the next chunk's included, at each mailbox take).
constexpr int kWaitVm0 = 0x0f70;
__device__ __forceinline__ void lists_settled() { __builtin_amdgcn_s_waitcnt(kWaitVm0); }

// Pair q of chunk k (steps k CK + 2q and the next) holds a step of the lane's
// walk [lo, hi).  A pair of padding steps reads and writes the lane's 16
// bytes of the zero block instead of its walk slot: its operands are zeros
// (the carry and the stack skip padding, and products of zeros and finite
// values are zeros, so only zeros are written back), and a memory line of
// such pairs is never fetched from HBM.  The choice is an address select,
// not a branch, so that the loads of the next chunk stay in flight while
// this one is swept.
__device__ __forceinline__ bool pair_real(int k, int q, int lo, int hi) {
  const int t = k * CK + 2 * q;
  return t + 2 > lo && t < hi;
}
__device__ __forceinline__ const double2_t* pair_src(const double* a, int64_t o, bool real, const double2_t* zp) {
  return real ? (const double2_t*)a + o : zp;
}

template <int RHS>
__device__ __forceinline__ void step_load_b(StepChunk<RHS>& C, const CellLoop& L, const hines::KCellWave& W,
                                            const cflag_t* flv, int k, int lane, int lo, int hi,
                                            const double2_t* zp) {
  C.fl = flag_ld(flv + 64 * k);
  if constexpr (RHS == kFlowNoise)
    C.p = pos_ld((const u32x4*)(L.lp + (W.chunk_off + k) * hines::kCellChunkElems) + (CK / 8) * lane);
#pragma unroll
  for (int q = 0; q < CK / 2; ++q) {
    const int64_t o = walk_pair(W.chunk_off + k, q, lane);
    const bool real = pair_real(k, q, lo, hi);
    C.f[q] = *pair_src(L.f, o, real, zp);
    C.r[q] = *pair_src(L.r, o, real, zp);
    C.c[q] = *pair_src(L.c, o, real, zp);
    if constexpr (RHS == kFlowCVI) C.i[q] = *pair_src(L.ci, o, real, zp);
    C.v[q] = *pair_src(L.v, o, real, zp);
  }
}

template <int RHS>
__device__ __forceinline__ void step_load_f(StepChunk<RHS>& C, const CellLoop& L, const hines::KCellWave& W,
                                            const cflag_t* flv, int k, int lane, int lo, int hi,
                                            const double2_t* zp) {
  C.fl = flag_ld(flv + 64 * k);
#pragma unroll
  for (int q = 0; q < CK / 2; ++q) {
    const int64_t o = walk_pair(W.chunk_off + k, q, lane);
    const bool real = pair_real(k, q, lo, hi);
    C.f[q] = *pair_src(L.f, o, real, zp);
    C.v[q] = *pair_src(L.v, o, real, zp);  // y from the backward sweep
  }
}

template <int RHS>
__device__ __forceinline__ void step_backward(const StepChunk<RHS>& C, const CellLoop& L, const hines::KCellWave& W,
                                              int k, int lane, int lo, int hi, double2_t* zp, int64_t base,
                                              lds_f64* stk, lds_f64* mb, double& cb, double& tb, int& m,
                                              unsigned& msrc) {
  double y[CK];
#pragma unroll
  for (int e = 0; e < CK; ++e) {
    const unsigned fe = cell_byte(C.fl, e);
    double bb = pair_at(C.c, e) * pair_at(C.v, e);
    if constexpr (RHS == kFlowCVI) bb = bb + pair_at(C.i, e);
    if constexpr (RHS == kFlowNoise) {
      const unsigned p = cell_pos(C.p, e);
      bb = bb + noise_draw(L.seed, L.step, (uint64_t)(base + (p == hines::kCellPadPos ? 0u : p)), L.sigma);
    }
    const double kc = (fe & hines::CF_TIP) ? 0.0 : 1.0;
    bb = __builtin_fma(-kc, cb, bb);
    if (fe & hines::CF_MBIN) {
      bb = bb - mb[msrc & 63u];
      msrc >>= 6;
    }
    if (fe & hines::CF_POP) {
      bb = bb - tb;
      m -= 1;
      tb = stk[64 * m];
    }
    y[e] = bb * pair_at(C.r, e);
    cb = pair_at(C.f, e) * bb;
    if (fe & hines::CF_PUSH) {
      stk[64 * m] = tb;
      m += 1;
      tb = cb;
    }
    if (fe & hines::CF_MERGE) tb = tb + cb;
    if (fe & hines::CF_MBOUT) mb[lane] = cb;
    if (e & 1) {
      const bool real = pair_real(k, e >> 1, lo, hi);
      *(real ? (double2_t*)L.v + walk_pair(W.chunk_off + k, e >> 1, lane) : zp) = double2_t{y[e - 1], y[e]};
    }
  }
}

template <int RHS>
__device__ __forceinline__ void step_forward(const StepChunk<RHS>& C, const CellLoop& L, const hines::KCellWave& W,
                                             int k, int lane, int lo, int hi, double2_t* zp, lds_f64* stk,
                                             lds_f64* mb, double& xc, double& xt, int& m, unsigned& msrc) {
  double x[CK];
#pragma unroll
  for (int e = CK - 1; e >= 0; --e) {
    const unsigned fe = cell_byte(C.fl, e);
    double xp = (fe & (hines::CF_PUSH | hines::CF_MERGE)) ? xt : xc;
    if (fe & hines::CF_MBOUT) xp = mb[lane];
    if (fe & hines::CF_PUSH) {
      m -= 1;
      xt = stk[64 * m];
    }
    const double xv = __builtin_fma(-pair_at(C.f, e), xp, pair_at(C.v, e));
    if (fe & hines::CF_POP) {
      stk[64 * m] = xt;
      m += 1;
      xt = xv;
    }
    if (fe & hines::CF_MBIN) {
      mb[msrc & 63u] = xv;
      msrc >>= 6;
    }
    xc = xv;
    x[e] = xv;
    if (!(e & 1)) {
      const bool real = pair_real(k, e >> 1, lo, hi);
      *(real ? (double2_t*)L.v + walk_pair(W.chunk_off + k, e >> 1, lane) : zp) = double2_t{x[e], x[e + 1]};
    }
  }
}

template <int RHS>
__global__ __launch_bounds__(64) void k_cells_step(DevTables tb, CellLoop L) {
  __shared__ __attribute__((aligned(16))) double sraw[hines::kCellStack * 64 + 64];
  lds_f64* stk = (lds_f64*)sraw + threadIdx.x;  // slot s at stk[64 s]
  lds_f64* mb = (lds_f64*)sraw + hines::kCellStack * 64;
  const int lane = threadIdx.x;
  const hines::KCellWave W = tb.cwave[blockIdx.x];
  const int nk = W.nchunk;
  const cflag_t* flv = (const cflag_t*)(tb.cflag + W.chunk_off * hines::kCellChunkElems) + lane;
  int64_t base = 0;
  if constexpr (RHS == kFlowNoise) base = tb.cbase[(int64_t)blockIdx.x * 64 + lane];
  StepChunk<RHS> A, B;
  const uint64_t ms = tb.cmsrc[(int64_t)blockIdx.x * 64 + lane];
  unsigned msb = (unsigned)ms, msf = (unsigned)(ms >> 32);
  const uint64_t rg = tb.crange[(int64_t)blockIdx.x * 64 + lane];
  const int lo = (int)(unsigned)rg, hi = (int)(unsigned)(rg >> 32);
  double2_t* zp = (double2_t*)tb.czero + lane;
  lists_settled();
  // backward: y = (b - contributions) / d', in place of V
  double cb = 0.0, tb_ = 0.0;
  int m = 0;
  // the next chunk is loaded unconditionally (past the end, the last chunk
  // again, unused): loads under a branch would make the compiler wait for
  // every load in flight where the branches join
  step_load_b<RHS>(A, L, W, flv, 0, lane, lo, hi, zp);
  for (int k = 0;; k += 2) {
    step_load_b<RHS>(B, L, W, flv, min(k + 1, nk - 1), lane, lo, hi, zp);
    step_backward<RHS>(A, L, W, k, lane, lo, hi, zp, base, stk, mb, cb, tb_, m, msb);
    if (k + 1 >= nk) break;
    step_load_b<RHS>(A, L, W, flv, min(k + 2, nk - 1), lane, lo, hi, zp);
    step_backward<RHS>(B, L, W, k + 1, lane, lo, hi, zp, base, stk, mb, cb, tb_, m, msb);
    if (k + 2 >= nk) break;
  }
  // the forward sweep reads back this wave's own stores
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  double xc = 0.0, xt = 0.0;
  m = 0;
  step_load_f<RHS>(A, L, W, flv, nk - 1, lane, lo, hi, zp);
  for (int k = nk - 1;; k -= 2) {
    step_load_f<RHS>(B, L, W, flv, max(k - 1, 0), lane, lo, hi, zp);
    step_forward<RHS>(A, L, W, k, lane, lo, hi, zp, stk, mb, xc, xt, m, msf);
    if (k < 1) break;
    step_load_f<RHS>(A, L, W, flv, max(k - 2, 0), lane, lo, hi, zp);
    step_forward<RHS>(B, L, W, k - 1, lane, lo, hi, zp, stk, mb, xc, xt, m, msf);
    if (k < 2) break;
  }
}

// ---------------------------------------------------------------------------
// Solve in the walk layout (cell-lane plans; paper §7, Fig 7.1: the solver
// works on its own data format, permutation kernels move data into and out
// of it).  d, u, b and x sit in the walk layout of k_cells_to_walk, so every
// access of the sweeps is one coalesced 16-byte unit per lane (a KiB per wave
// instruction) and no gather passes through LDS.  The elimination is the
// cell-lane one (cell_backward's flags, stack and mailboxes); the backward
// sweep stores f = u / d' in the plan's scratch and y = b' / d' in x, the
// forward sweep overwrites y with x.  Roots and padding have no coupling.
// ---------------------------------------------------------------------------
struct WalkSolve {
  const double* d;
  const double* u;
  const double* b;
  double* x;
  double* f;  // f per walk slot (the plan's scratch)
};

struct WalkChunk {
  double2_t d[CK / 2], u[CK / 2], b[CK / 2];
  cflag_t fl;
};

__device__ __forceinline__ void walk_load_b(WalkChunk& C, const WalkSolve& L, const cflag_t* flv, int64_t chunk,
                                            int k, int lane) {
  C.fl = flag_ld(flv + 64 * k);
#pragma unroll
  for (int q = 0; q < CK / 2; ++q) {
    const int64_t o = walk_pair(chunk, q, lane);
    C.d[q] = ((const double2_t*)L.d)[o];
    C.u[q] = ((const double2_t*)L.u)[o];
    C.b[q] = ((const double2_t*)L.b)[o];
  }
}

__device__ __forceinline__ void walk_load_f(WalkChunk& C, const WalkSolve& L, const cflag_t* flv, int64_t chunk,
                                            int k, int lane) {
  C.fl = flag_ld(flv + 64 * k);
#pragma unroll
  for (int q = 0; q < CK / 2; ++q) {
    const int64_t o = walk_pair(chunk, q, lane);
    C.d[q] = ((const double2_t*)L.f)[o];  // f
    C.b[q] = ((const double2_t*)L.x)[o];  // y
  }
}

__device__ __forceinline__ void walk_backward(const WalkChunk& C, const WalkSolve& L, int64_t chunk, int lane,
                                              lds_d2* stk, lds_d2* mb, double& cd, double& cb, double& td,
                                              double& tb, int& m, unsigned& msrc) {
  double fv[CK], yv[CK];
#pragma unroll
  for (int e = 0; e < CK; ++e) {
    const unsigned fe = cell_byte(C.fl, e);
    double dd = pair_at(C.d, e), bb = pair_at(C.b, e);
    const double uu = (fe & (hines::CF_ROOT | hines::CF_PAD)) ? 0.0 : pair_at(C.u, e);
    const double kc = (fe & hines::CF_TIP) ? 0.0 : 1.0;
    dd = __builtin_fma(-kc, cd, dd);
    bb = __builtin_fma(-kc, cb, bb);
    if (fe & hines::CF_MBIN) {
      const double2_t mv = mb[msrc & 63u];
      msrc >>= 6;
      dd = dd - mv.x;
      bb = bb - mv.y;
    }
    if (fe & hines::CF_POP) {
      dd = dd - td;
      bb = bb - tb;
      m -= 1;
      const double2_t t = stk[64 * m];
      td = t.x;
      tb = t.y;
    }
    const double rr = rcp_nr(dd);
    fv[e] = uu * rr;
    yv[e] = bb * rr;
    cd = uu * fv[e];
    cb = fv[e] * bb;
    if (fe & hines::CF_PUSH) {
      stk[64 * m] = double2_t{td, tb};
      m += 1;
      td = cd;
      tb = cb;
    }
    if (fe & hines::CF_MERGE) {
      td = td + cd;
      tb = tb + cb;
    }
    if (fe & hines::CF_MBOUT) mb[lane] = double2_t{cd, cb};
  }
#pragma unroll
  for (int q = 0; q < CK / 2; ++q) {
    const int64_t o = walk_pair(chunk, q, lane);
    ((double2_t*)L.f)[o] = double2_t{fv[2 * q], fv[2 * q + 1]};
    ((double2_t*)L.x)[o] = double2_t{yv[2 * q], yv[2 * q + 1]};
  }
}

__device__ __forceinline__ void walk_forward(const WalkChunk& C, const WalkSolve& L, int64_t chunk, int lane,
                                             lds_f64* stx, lds_d2* mb, double& xc, double& xt, int& m,
                                             unsigned& msrc) {
  double x[CK];
#pragma unroll
  for (int e = CK - 1; e >= 0; --e) {
    const unsigned fe = cell_byte(C.fl, e);
    double xp = (fe & (hines::CF_PUSH | hines::CF_MERGE)) ? xt : xc;
    if (fe & hines::CF_MBOUT) xp = mb[lane].x;  // x of the parent, posted by the receiving lane
    if (fe & hines::CF_PUSH) {
      m -= 1;
      xt = stx[64 * m];
    }
    const double xv = __builtin_fma(-pair_at(C.d, e), xp, pair_at(C.b, e));
    if (fe & hines::CF_POP) {
      stx[64 * m] = xt;
      m += 1;
      xt = xv;
    }
    if (fe & hines::CF_MBIN) {
      mb[msrc & 63u].x = xv;
      msrc >>= 6;
    }
    xc = xv;
    x[e] = xv;
  }
#pragma unroll
  for (int q = 0; q < CK / 2; ++q)
    ((double2_t*)L.x)[walk_pair(chunk, q, lane)] = double2_t{x[2 * q], x[2 * q + 1]};
}

__global__ __launch_bounds__(64) void k_solve_walk(DevTables tb, WalkSolve L) {
  __shared__ __attribute__((aligned(16))) double2_t wraw[hines::kCellStack * 64 + 64];
  lds_d2* stk = (lds_d2*)wraw + threadIdx.x;  // slot s at stk[64 s]
  lds_d2* mb = (lds_d2*)wraw + hines::kCellStack * 64;
  const int lane = threadIdx.x;
  const hines::KCellWave W = tb.cwave[blockIdx.x];
  const int nk = W.nchunk;
  const cflag_t* flv = (const cflag_t*)(tb.cflag + W.chunk_off * hines::kCellChunkElems) + lane;
  WalkChunk A, B;
  const uint64_t ms = tb.cmsrc[(int64_t)blockIdx.x * 64 + lane];
  unsigned msb = (unsigned)ms, msf = (unsigned)(ms >> 32);
  double cd = 0.0, cb = 0.0, td = 0.0, tb_ = 0.0;
  int m = 0;
  walk_load_b(A, L, flv, W.chunk_off, 0, lane);
  for (int k = 0;; k += 2) {
    if (k + 1 < nk) walk_load_b(B, L, flv, W.chunk_off + k + 1, k + 1, lane);
    walk_backward(A, L, W.chunk_off + k, lane, stk, mb, cd, cb, td, tb_, m, msb);
    if (k + 1 >= nk) break;
    if (k + 2 < nk) walk_load_b(A, L, flv, W.chunk_off + k + 2, k + 2, lane);
    walk_backward(B, L, W.chunk_off + k + 1, lane, stk, mb, cd, cb, td, tb_, m, msb);
    if (k + 2 >= nk) break;
  }
  // the forward sweep reads back this wave's own stores
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  lds_f64* stx = (lds_f64*)wraw + threadIdx.x;  // slot s at stx[64 s]
  double xc = 0.0, xt = 0.0;
  m = 0;
  walk_load_f(A, L, flv, W.chunk_off + nk - 1, nk - 1, lane);
  for (int k = nk - 1;; k -= 2) {
    if (k >= 1) walk_load_f(B, L, flv, W.chunk_off + k - 1, k - 1, lane);
    walk_forward(A, L, W.chunk_off + k, lane, stx, mb, xc, xt, m, msf);
    if (k < 1) break;
    if (k >= 2) walk_load_f(A, L, flv, W.chunk_off + k - 2, k - 2, lane);
    walk_forward(B, L, W.chunk_off + k - 1, lane, stx, mb, xc, xt, m, msf);
    if (k < 2) break;
  }
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

  dma16<T>(tb.br + G.br_begin, lds_raw + L.br_off_bytes(), G.nbr, tid);
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

// Row test of strict diagonal dominance with a positive diagonal (paper §1):
// d_i > |u_i| (non-root) + sum over children k of |u_k|, children in ascending
// order.  A failing row lowers *bad to its index (NaN rows fail).
__global__ void k_check_sdd(int64_t n, const int32_t* __restrict__ parent, const int32_t* __restrict__ ch_off,
                            const int32_t* __restrict__ ch, const double* __restrict__ d,
                            const double* __restrict__ u, unsigned long long* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = parent[i] >= 0 ? fabs(u[i]) : 0.0;
  for (int32_t k = ch_off[i]; k < ch_off[i + 1]; ++k) s += fabs(u[ch[k]]);
  if (!(d[i] > s)) atomicMin(bad, (unsigned long long)i);
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
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
