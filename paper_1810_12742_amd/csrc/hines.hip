// MI355X (gfx950) batched Hines solver: device tables, solve kernels and the
// C-ABI declared in include/hines.h.
//
// Design (paper §3-§5 re-thought for CDNA4):
//  * one workgroup solves one packed group of cells (§3: all work of a matrix
//    stays inside one block, so only block-level synchronisation is needed);
//  * the group's cells are contiguous user ranges: they are streamed from HBM
//    into LDS with fully coalesced loads, eliminated there, and the solution
//    is streamed back, so every matrix entry crosses HBM exactly once (the
//    role of the paper's interleaved layout, §5, is played by LDS);
//  * one lane per branch, level-synchronous sweeps (§3), lanes sorted by
//    branch length inside a level (§4, Fig 4.1);
//  * sibling branches never write the same parent compartment: each branch
//    stores its elimination contribution in its own LDS slot and the parent's
//    lane pulls its children's slots in a fixed order (no atomics, bitwise
//    reproducible);
//  * groups are bucketed by LDS footprint; one launch per bucket so the
//    per-CU occupancy follows the bucket's footprint.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/hines.h"
#include "setup.hpp"

using hines::KBranch;
using hines::KCell;
using hines::KGroup;

namespace {

thread_local std::string g_last_error;

hines_status set_err(hines_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

hines_status ok() {
  g_last_error.clear();
  return HINES_OK;
}

constexpr int kMaxLdsBytes = 160 * 1024;  // gfx950 LDS per workgroup

// LDS image of a group in the FP64 kernel: d, u, b per compartment, the two
// elimination contributions per branch, the branch records and the level
// offsets.  Every region starts 16-byte aligned.
struct LdsLayout {
  int32_t nunk, nbr_pad, nlev;
  __host__ __device__ int64_t u_off() const { return nunk; }  // in doubles
  __host__ __device__ int64_t b_off() const { return 2 * (int64_t)nunk; }
  __host__ __device__ int64_t cd_off() const { return 3 * (int64_t)nunk; }
  __host__ __device__ int64_t cb_off() const { return 3 * (int64_t)nunk + nbr_pad; }
  __host__ __device__ int64_t br_off_bytes() const { return 8 * (3 * (int64_t)nunk + 2 * (int64_t)nbr_pad); }
  __host__ __device__ int64_t seg_off_bytes() const { return br_off_bytes() + 16 * (int64_t)nbr_pad; }
  __host__ __device__ int64_t bytes() const {
    const int64_t ints = (int64_t)nlev + 1 > hines::kSchedLanes + 1 ? (int64_t)nlev + 1 : hines::kSchedLanes + 1;
    return (seg_off_bytes() + 4 * ints + 15) & ~(int64_t)15;
  }
};
__host__ __device__ inline LdsLayout lds_layout(const KGroup& g) { return LdsLayout{g.nunk, (g.nbr + 1) & ~1, g.nlev}; }
inline int64_t lds_bytes_f64(const KGroup& g) { return lds_layout(g).bytes(); }

// Footprint buckets (bytes).  A launch reserves its bucket's size per workgroup.
constexpr int kBuckets[] = {4096,  8192,  12288, 16384, 20480, 24576,  32768,  40960,
                            49152, 65536, 81920, 98304, 131072, 163840};

struct DevTables {
  const KBranch* br;    // lane order
  const KGroup* grp;    // per group
  const int32_t* seg;   // first lane of each (group, level) segment; nseg+1 entries
  const KCell* cell;    // group order
  const int32_t* glist; // group ids of one launch
  const int32_t* lanes; // scheduled plans: per group kSchedLanes + 1 record offsets
};

}  // namespace

struct hines_plan {
  hines::HostPlan host;
  int device = -1;
  void* dev_mem = nullptr;
  int64_t dev_bytes = 0;
  DevTables t{};
  struct Bucket {
    int32_t lds_bytes, first, count;
  };
  std::vector<Bucket> buckets;
  int64_t max_lds = 0;
};

// ---------------------------------------------------------------------------
// Group staging.  Compartments of a group are copied from HBM into the LDS
// image with 16-byte global->LDS DMA (two doubles per lane, 1 KiB per wave
// instruction), the branch records with one 16-byte record per lane and the
// level offsets with 4-byte DMA, so every load of a group is in flight at
// once without occupying registers.  A contiguous group (consecutive cells)
// is one aligned range; other groups are copied cell by cell.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void_t;

// Copy `pairs` 16-byte units from src to dst (both 16-byte aligned in LDS;
// the global side may be 8-byte aligned).
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

// Stage d, u, b of one user range [lo, lo + n) at LDS slot `slot` (even).
template <int T>
__device__ __forceinline__ void stage_range(const double* d, const double* u, const double* rhs, int64_t lo, int n,
                                            int slot, double* D, double* U, double* B, int tid) {
  const int units = n >> 1;
  dma16<T>(d + lo, D + slot, units, tid);
  dma16<T>(u + lo, U + slot, units, tid);
  dma16<T>(rhs + lo, B + slot, units, tid);
}

template <int T>
__device__ __forceinline__ void stage_group(const DevTables& tb, const KGroup& G, const LdsLayout& L,
                                            const double* d, const double* u, const double* rhs, char* lds,
                                            int tid, const int32_t* lane_table = nullptr) {
  double* D = (double*)lds;
  double* U = D + L.u_off();
  double* B = D + L.b_off();
  dma16<T>(tb.br + G.br_begin, lds + L.br_off_bytes(), G.nbr, tid);
  if (lane_table)
    dma4<T>(lane_table, lds + L.seg_off_bytes(), hines::kSchedLanes + 1, tid);
  else
    dma4<T>(tb.seg + G.seg_begin, lds + L.seg_off_bytes(), G.nlev + 1, tid);
  if (G.contig) {
    // slots kLdsPad + [0, user_lo + user_n) <-> user [user_base, ...); both ends 16-byte aligned
    const int span = G.user_lo + G.user_n;
    stage_range<T>(d, u, rhs, G.user_base, span & ~1, hines::kLdsPad, D, U, B, tid);
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    const bool tail = (span & 1) && tid == 0;
    if (tail) {
      const int64_t k = G.user_base + span - 1;
      t0 = d[k];
      t1 = u[k];
      t2 = rhs[k];
    }
    __builtin_amdgcn_s_waitcnt(0);
    if (tail) {
      D[hines::kLdsPad + span - 1] = t0;
      U[hines::kLdsPad + span - 1] = t1;
      B[hines::kLdsPad + span - 1] = t2;
    }
  } else {
    for (int c = 0; c < G.ncell; ++c) {
      const KCell C = tb.cell[G.cell_begin + c];
      stage_range<T>(d, u, rhs, C.user_lo, C.n, C.lds, D, U, B, tid);
      if ((C.n & 1) && tid == 0) {
        const int64_t k = C.user_lo + C.n - 1;
        const double t0 = d[k], t1 = u[k], t2 = rhs[k];
        D[C.lds + C.n - 1] = t0;
        U[C.lds + C.n - 1] = t1;
        B[C.lds + C.n - 1] = t2;
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();
}

template <int T>
__device__ __forceinline__ void store_range(const double* B, int slot, double* x, int64_t lo, int n, int tid) {
  // 16-byte LDS reads and global stores for the pairs, then the odd element
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
    // the user range starts at slot kLdsPad + user_lo (user_lo 0 or 1); store
    // slot-aligned pairs from the first even slot, then the edges
    const int lo = G.user_lo, hi = G.user_lo + G.user_n;
    const int a = (lo + 1) & ~1;  // first even offset at or after lo
    const double* Bp = B + hines::kLdsPad;
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
// second-order Newton step, r1 = r0 (1 + e + e^2) with e = 1 - d r0, whose
// error e^3 is below double rounding.
__device__ __forceinline__ double rcp_nr(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  const double e = __builtin_fma(-d, r, 1.0);
  const double t = __builtin_fma(e, e, e);
  return __builtin_fma(r, t, r);
}

constexpr int kChunk = 8;  // compartments held in registers per LDS round trip

// ---------------------------------------------------------------------------
// FP64 solve of one group in LDS (paper §2 Listing 2, §3 level-synchronous
// sweeps).  Branch with compartments p_0 (root side) ... p_{len-1}; u_j is
// the coupling of p_j to p_{j-1} (at p_j for a branch running toward higher
// user indices, at p_{j-1}, the old child, for one running toward lower ones
// after re-rooting); the pull subtracts the children's contributions in
// descending order of their first user index.
//
// Fast form (default).  Backward, levels deepest -> 0:
//   r_j = 1/d'_j, f_j = u_j r_j, y_j = b'_j r_j  (stored in place of d_j, b_j)
//   d'_{j-1} = d_{j-1} - f_j u_j,  b'_{j-1} = b_{j-1} - f_j b'_j
//   j = 0: root: x = b' r; otherwise the contribution (f_0 u_0, f_0 b'_0)
//   goes to the branch's own slot.
// Forward, levels 0 -> deepest: x_j = y_j - f_j x_{j-1} (x_{-1}: the parent
// compartment's solution), one fused multiply-add per compartment.
// Each branch is walked in chunks of kChunk compartments whose operands are
// fetched from LDS together, so the dependent chain runs out of registers.
//
// Bitwise form: the plain algorithm's operations (IEEE division, separately
// rounded multiply and subtract) in its order, so the solution equals the
// plain algorithm on the plan numbering bit for bit.
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

// Ascending branches (no re-rooting): compartment j of a branch sits at LDS
// slot start + j, so a chunk of 8 positions is a fixed window addressed from
// one base with immediate offsets.  The window may reach 8 slots beyond the
// branch (into the padding or other branches); those values are never used
// and nothing outside the branch is written.
__device__ __forceinline__ void backward_asc(const KBranch br, double* D, const double* U, double* B, double* CD,
                                             double* CB) {
  const int len = br.lendir;
  int i = br.start + len - 1;
  double dl = D[i], bl = B[i];
  for (int k = br.nchild - 1; k >= 0; --k) {
    dl = dl - CD[br.child0 + k];
    bl = bl - CB[br.child0 + k];
  }
  int rem = len - 1;
  while (rem > 0) {
    const int n = rem < kChunk ? rem : kChunk;
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
    rem -= n;
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

__device__ __forceinline__ void forward_asc(const KBranch br, const double* D, double* B) {
  const int len = br.lendir;
  int i = br.start;
  double xp;
  if (br.u0 >= 0) {
    xp = __builtin_fma(-D[i], B[br.pslot], B[i]);
    B[i] = xp;
  } else {
    xp = B[i];
  }
  int rem = len - 1;
  while (rem > 0) {
    const int n = rem < kChunk ? rem : kChunk;
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

template <int T, int MODE>
__global__ __launch_bounds__(T) void k_solve_lds_f64(DevTables tb, const double* __restrict__ d,
                                                     const double* __restrict__ u, const double* rhs,
                                                     double* x) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  const int g = tb.glist[blockIdx.x];
  const KGroup G = tb.grp[g];
  const LdsLayout L = lds_layout(G);
  double* D = (double*)lds_raw;
  double* U = D + L.u_off();
  double* B = D + L.b_off();
  double* CD = D + L.cd_off();
  double* CB = D + L.cb_off();
  const KBranch* BR = (const KBranch*)(lds_raw + L.br_off_bytes());
  const int* seg = (const int*)(lds_raw + L.seg_off_bytes());
  const int tid = threadIdx.x;
  const int brb = G.br_begin;

  stage_group<T>(tb, G, L, d, u, rhs, lds_raw, tid);

  // Backward sweep; the first record of the next level is fetched while the
  // current level runs (records are never written after staging).
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

  // Forward sweep, levels 0 -> deepest.
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
// Scheduled FP64 solve (ascending branches, fast form).  One wave per group;
// lane t runs the branches the setup assigned to it, each starting at its
// scheduled iteration.  In one iteration a lane eliminates up to kSchedChunk
// compartments of its current branch; a branch starts only after every child
// branch finished in an earlier iteration, so its children's contributions
// are in LDS.  The forward sweep replays the schedule backwards in time: a
// branch's parent compartment is solved in a later backward iteration, hence
// in an earlier forward one.  No barrier is needed between iterations: the
// group is one wave and the LDS executes a wave's operations in order; the
// signal fence only keeps the compiler from moving LDS accesses across
// iterations.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int sched_itlen(int len) {
  const int k = (len - 1 + hines::kSchedChunk - 1) / hines::kSchedChunk;
  return k > 1 ? k : 1;
}

__global__ __launch_bounds__(64) void k_solve_sched_f64(DevTables tb, const double* __restrict__ d,
                                                        const double* __restrict__ u, const double* rhs,
                                                        double* x) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  const int g = tb.glist[blockIdx.x];
  const KGroup G = tb.grp[g];
  const LdsLayout L = lds_layout(G);
  double* D = (double*)lds_raw;
  double* U = D + L.u_off();
  double* B = D + L.b_off();
  double* CD = D + L.cd_off();
  double* CB = D + L.cb_off();
  const KBranch* BR = (const KBranch*)(lds_raw + L.br_off_bytes());
  const int* LO = (const int*)(lds_raw + L.seg_off_bytes());
  const int lane = threadIdx.x;

  stage_group<64>(tb, G, L, d, u, rhs, lds_raw, lane, tb.lanes + (int64_t)g * (hines::kSchedLanes + 1));

  const int q0 = LO[lane], q1 = LO[lane + 1];
  const int F = G.makespan;

  // ---- backward ----
  {
    int q = q0;
    KBranch rec{};
    int js = 0x7fffffff;
    if (q < q1) {
      rec = BR[q];
      js = rec.pad;
    }
    int i = 0, rem = -1;
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
          const double* pd = D + (i - kChunk);
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
          rem -= n;
        }
        if (rem == 0) {
          const double r = rcp_nr(dl);
          if (rec.u0 >= 0) {
            const double uu = U[rec.u0];
            const double f = uu * r;
            D[i] = f;
            B[i] = bl * r;
            CD[rec.self] = f * uu;
            CB[rec.self] = f * bl;
          } else {
            B[i] = bl * r;
          }
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

  // ---- forward: the same schedule, backwards in time ----
  {
    int q = q1 - 1;
    KBranch rec{};
    int je = -1;
    if (q >= q0) {
      rec = BR[q];
      je = rec.pad + sched_itlen(rec.lendir) - 1;
    }
    int i = 0, rem = -1;
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

namespace {

template <int T, int MODE>
hipError_t launch_solve_f64(const hines_plan* p, const double* d, const double* u, const double* b, double* x,
                            hipStream_t s) {
  for (const auto& bk : p->buckets) {
    if (bk.count == 0) continue;
    DevTables t = p->t;
    t.glist = p->t.glist + bk.first;
    hipLaunchKernelGGL((k_solve_lds_f64<T, MODE>), dim3(bk.count), dim3(T), bk.lds_bytes, s, t, d, u, b, x);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int T>
hipError_t allow_lds_f64() {
  const void* fns[] = {(const void*)k_solve_lds_f64<T, kModeFast>, (const void*)k_solve_lds_f64<T, kModeBitwise>,
                       (const void*)k_solve_lds_f64<T, kModeAscending>};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t allow_lds(int T) {
  hipError_t e0 = hipFuncSetAttribute((const void*)k_solve_sched_f64, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      kMaxLdsBytes);
  if (e0 != hipSuccess) return e0;
  switch (T) {
    case 64: return allow_lds_f64<64>();
    case 128: return allow_lds_f64<128>();
    case 256: return allow_lds_f64<256>();
    case 512: return allow_lds_f64<512>();
    case 1024: return allow_lds_f64<1024>();
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sched_f64(const hines_plan* p, const double* d, const double* u, const double* b, double* x,
                            hipStream_t s) {
  for (const auto& bk : p->buckets) {
    if (bk.count == 0) continue;
    DevTables t = p->t;
    t.glist = p->t.glist + bk.first;
    hipLaunchKernelGGL(k_solve_sched_f64, dim3(bk.count), dim3(64), bk.lds_bytes, s, t, d, u, b, x);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int T>
hipError_t launch_f64(const hines_plan* p, const double* d, const double* u, const double* b, double* x,
                      hipStream_t s) {
  if (p->host.scheduled) return launch_sched_f64(p, d, u, b, x, s);
  if (p->host.opt.bitwise) return launch_solve_f64<T, kModeBitwise>(p, d, u, b, x, s);
  if (p->host.all_ascending) return launch_solve_f64<T, kModeAscending>(p, d, u, b, x, s);
  return launch_solve_f64<T, kModeFast>(p, d, u, b, x, s);
}

// Every index a kernel derives from the tables must stay inside the group's
// LDS image; checked once on the host before anything is uploaded.
bool check_kernel_tables(const hines::HostPlan& P, std::string& why) {
  if (!P.kernel_tables_fit) {
    why = "a group exceeds the int16 branch records";
    return false;
  }
  for (int64_t g = 0; g < P.ngroups; ++g) {
    const KGroup& G = P.kgroup[g];
    if (G.seg_begin < 0 || G.seg_begin + G.nlev + 1 > (int64_t)P.kseg.size() || G.br_begin != P.kseg[G.seg_begin] ||
        P.kseg[G.seg_begin + G.nlev] - G.br_begin != G.nbr) {
      why = "segment range";
      return false;
    }
    const int64_t pad = hines::kLdsPad;
    int64_t U = pad;
    if (G.contig) {
      if ((G.user_base & 1) || G.user_base < 0 || G.user_lo < 0 || G.user_lo > 1 ||
          G.user_base + G.user_lo + G.user_n > P.n) {
        why = "contiguous group range";
        return false;
      }
      U = pad + G.user_lo;
    }
    for (int c = 0; c < G.ncell; ++c) {
      const KCell& C = P.kcell[G.cell_begin + c];
      bool good = C.n > 0 && C.user_lo >= 0 && C.user_lo + C.n <= P.n;
      if (G.contig)
        good = good && C.lds == U && C.user_lo == G.user_base + C.lds - pad;
      else
        good = good && C.lds >= U && C.lds <= U + 1 && !(C.lds & 1);
      if (!good) {
        why = "cell table";
        return false;
      }
      U = C.lds + C.n;
    }
    if (G.contig && U != pad + G.user_lo + G.user_n) {
      why = "contiguous group size";
      return false;
    }
    if (G.nunk < U + pad || G.nunk > U + pad + 1 || (G.nunk & 1)) {
      why = "group size";
      return false;
    }
    for (int l = 0; l < G.nlev; ++l)
      for (int e = P.kseg[G.seg_begin + l]; e < P.kseg[G.seg_begin + l + 1]; ++e) {
        const KBranch& B = P.kbranch[e];
        int len = B.lendir > 0 ? B.lendir : -B.lendir;
        int dir = B.lendir > 0 ? 1 : -1;
        int last = B.start + dir * (len - 1);
        bool good = len >= 1 && B.start >= pad && B.start < U && last >= pad && last < U && B.self >= 0 &&
                    B.self < G.nbr && B.nchild >= 0 && (B.nchild == 0 || (B.child0 >= 0 && B.child0 + B.nchild <= G.nbr));
        if (B.u0 >= 0 || B.pslot >= 0) good = good && B.u0 >= pad && B.u0 < U && B.pslot >= pad && B.pslot < U;
        if (P.all_ascending && dir < 0) good = false;
        if (!good) {
          why = "branch table";
          return false;
        }
      }
  }
  if (P.scheduled) {
    // lanes' branches must not overlap in time and every branch must start
    // after its children finished; everything inside the makespan
    const int W = hines::kSchedLanes;
    if ((int64_t)P.klane.size() != P.ngroups * (W + 1)) {
      why = "lane table size";
      return false;
    }
    std::vector<int32_t> st, fin;
    for (int64_t g = 0; g < P.ngroups; ++g) {
      const KGroup& G = P.kgroup[g];
      const int32_t* lo = &P.klane[g * (W + 1)];
      if (lo[0] != 0 || lo[W] != G.nbr || G.makespan <= 0 || G.makespan > 30000) {
        why = "lane offsets";
        return false;
      }
      st.assign(G.nbr, -1);
      fin.assign(G.nbr, -1);
      for (int ln = 0; ln < W; ++ln) {
        if (lo[ln + 1] < lo[ln]) {
          why = "lane offsets order";
          return false;
        }
        int32_t t = 0;
        for (int32_t r = lo[ln]; r < lo[ln + 1]; ++r) {
          const KBranch& B = P.kbranch[G.br_begin + r];
          const int len = B.lendir;
          const int itl = std::max(1, (len - 1 + hines::kSchedChunk - 1) / hines::kSchedChunk);
          if (B.pad < t || B.pad + itl > G.makespan || B.self < 0 || B.self >= G.nbr || st[B.self] >= 0) {
            why = "lane timeline";
            return false;
          }
          st[B.self] = B.pad;
          fin[B.self] = B.pad + itl;
          t = B.pad + itl;
        }
      }
      for (int32_t r = 0; r < G.nbr; ++r) {
        const KBranch& B = P.kbranch[G.br_begin + r];
        for (int c = B.child0; c < B.child0 + B.nchild; ++c)
          if (st[c] < 0 || fin[c] > st[B.self]) {
            why = "schedule order";
            return false;
          }
      }
    }
  }
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
extern "C" {

void hines_default_options(hines_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof *opt);
  opt->group_width = 64;
  opt->max_group_unknowns = 2048;
  opt->keep_tables = 1;
}

hines_status hines_setup(const int32_t* parent, int64_t n, const int64_t* branch_offsets, int64_t nbranches,
                         const int64_t* cell_offsets, int32_t ncells, const hines_options* opt_in,
                         hines_plan** out) {
  if (!out) return set_err(HINES_ERR_NULL, "out is NULL");
  *out = nullptr;
  hines_options opt;
  if (opt_in)
    opt = *opt_in;
  else
    hines_default_options(&opt);
  for (int k = 0; k < 7; ++k)
    if (opt.reserved[k] != 0) return set_err(HINES_ERR_OPTION, "reserved option fields must be 0");
  hines::Options o;
  o.rebalance_root = opt.rebalance_root != 0;
  o.split_branches = opt.split_branches != 0;
  o.group_width = opt.group_width;
  o.cell_order = opt.cell_order;
  o.max_group_unknowns = opt.max_group_unknowns;
  o.host_only = opt.host_only != 0;
  o.keep_tables = opt.keep_tables != 0;
  o.bitwise = opt.bitwise != 0;
  o.scheduler = opt.level_sync ? 0 : 1;
  hines_plan* p = new (std::nothrow) hines_plan();
  if (!p) return set_err(HINES_ERR_OOM, "host allocation failed");
  std::string why;
  hines::Status s = hines::build_plan(parent, n, branch_offsets, nbranches, cell_offsets, ncells, o, p->host, why);
  if (s != hines::OK) {
    delete p;
    return set_err((hines_status)s, "%s", why.c_str());
  }
  if (!o.host_only && !check_kernel_tables(p->host, why)) {
    const hines_status st = p->host.kernel_tables_fit ? HINES_ERR_STATE : HINES_ERR_TOO_BIG;
    delete p;
    return set_err(st, "kernel tables: %s", why.c_str());
  }
  // LDS buckets
  const hines::HostPlan& P = p->host;
  const int nbk = (int)(sizeof kBuckets / sizeof kBuckets[0]);
  std::vector<std::vector<int32_t>> members(nbk);
  for (int64_t g = 0; g < P.ngroups; ++g) {
    int64_t bytes = lds_bytes_f64(P.kgroup[g]);
    p->max_lds = std::max(p->max_lds, bytes);
    int k = 0;
    while (k < nbk && kBuckets[k] < bytes) ++k;
    if (k == nbk) {
      if (!o.host_only) {
        int64_t gu = P.kgroup[g].nunk;
        delete p;
        return set_err(HINES_ERR_TOO_BIG, "group of %lld compartments needs %lld bytes of LDS (max %d)",
                       (long long)gu, (long long)bytes, kMaxLdsBytes);
      }
      k = nbk - 1;
    }
    members[k].push_back((int32_t)g);
  }
  std::vector<int32_t> glist;
  for (int k = 0; k < nbk; ++k) {
    auto& m = members[k];
    // longest critical path first (§4 balance: start the slow groups early)
    std::stable_sort(m.begin(), m.end(),
                     [&](int32_t a, int32_t b) { return P.kgroup[a].cost > P.kgroup[b].cost; });
    p->buckets.push_back({kBuckets[k], (int32_t)glist.size(), (int32_t)m.size()});
    glist.insert(glist.end(), m.begin(), m.end());
  }
  if (o.host_only) {
    *out = p;
    return ok();
  }
  // upload: one allocation, 256-byte aligned sub-buffers
  auto al = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
  const int64_t sz_br = al((int64_t)P.kbranch.size() * sizeof(KBranch));
  const int64_t sz_grp = al((int64_t)P.kgroup.size() * sizeof(KGroup));
  const int64_t sz_seg = al((int64_t)P.kseg.size() * sizeof(int32_t));
  const int64_t sz_cell = al((int64_t)P.kcell.size() * sizeof(KCell));
  const int64_t sz_gl = al((int64_t)glist.size() * sizeof(int32_t));
  const int64_t sz_ln = al((int64_t)P.klane.size() * sizeof(int32_t));
  const int64_t total = sz_br + sz_grp + sz_seg + sz_cell + sz_gl + sz_ln + 256;
  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) e = allow_lds(o.group_width);
  if (e != hipSuccess) {
    delete p;
    return set_err(HINES_ERR_HIP, "device setup: %s", hipGetErrorString(e));
  }
  e = hipMalloc(&p->dev_mem, total);
  if (e != hipSuccess) {
    p->dev_mem = nullptr;
    delete p;
    return set_err(HINES_ERR_OOM, "hipMalloc(%lld): %s", (long long)total, hipGetErrorString(e));
  }
  p->dev_bytes = total;
  char* base = (char*)p->dev_mem;
  auto up = [&](const void* src, int64_t bytes, int64_t slot) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpy(base + slot, src, bytes, hipMemcpyHostToDevice);
  };
  int64_t off = 0;
  p->t.br = (const KBranch*)(base + off);
  e = up(P.kbranch.data(), (int64_t)P.kbranch.size() * sizeof(KBranch), off);
  off += sz_br;
  p->t.grp = (const KGroup*)(base + off);
  if (e == hipSuccess) e = up(P.kgroup.data(), (int64_t)P.kgroup.size() * sizeof(KGroup), off);
  off += sz_grp;
  p->t.seg = (const int32_t*)(base + off);
  if (e == hipSuccess) e = up(P.kseg.data(), (int64_t)P.kseg.size() * sizeof(int32_t), off);
  off += sz_seg;
  p->t.cell = (const KCell*)(base + off);
  if (e == hipSuccess) e = up(P.kcell.data(), (int64_t)P.kcell.size() * sizeof(KCell), off);
  off += sz_cell;
  p->t.glist = (const int32_t*)(base + off);
  if (e == hipSuccess) e = up(glist.data(), (int64_t)glist.size() * sizeof(int32_t), off);
  off += sz_gl;
  p->t.lanes = P.scheduled ? (const int32_t*)(base + off) : nullptr;
  if (e == hipSuccess && P.scheduled) e = up(P.klane.data(), (int64_t)P.klane.size() * sizeof(int32_t), off);
  if (e != hipSuccess) {
    hipFree(p->dev_mem);
    delete p;
    return set_err(HINES_ERR_HIP, "table upload: %s", hipGetErrorString(e));
  }
  // the kernel tables now live on the device
  std::vector<KBranch>().swap(p->host.kbranch);
  *out = p;
  return ok();
}

hines_status hines_solve(const hines_plan* p, const double* diag, const double* upper, const double* rhs, double* x,
                         int32_t ncells, void* stream) {
  if (!p) return set_err(HINES_ERR_NULL, "plan is NULL");
  if (p->host.opt.host_only) return set_err(HINES_ERR_STATE, "plan was built host_only");
  if (ncells != p->host.ncells) return set_err(HINES_ERR_NCELLS, "ncells %d != plan's %lld", ncells, (long long)p->host.ncells);
  if (p->host.n == 0) return ok();
  if (!diag || !upper || !rhs || !x) return set_err(HINES_ERR_NULL, "a device array is NULL");
  if ((const void*)x == (const void*)diag || (const void*)x == (const void*)upper)
    return set_err(HINES_ERR_STATE, "x must not alias diag or upper");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return set_err(HINES_ERR_STATE, "current device %d is not the plan's device %d", dev, p->device);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  switch (p->host.opt.group_width) {
    case 64: e = launch_f64<64>(p, diag, upper, rhs, x, s); break;
    case 128: e = launch_f64<128>(p, diag, upper, rhs, x, s); break;
    case 256: e = launch_f64<256>(p, diag, upper, rhs, x, s); break;
    case 512: e = launch_f64<512>(p, diag, upper, rhs, x, s); break;
    default: e = launch_f64<1024>(p, diag, upper, rhs, x, s); break;
  }
  if (e != hipSuccess) return set_err(HINES_ERR_HIP, "launch: %s", hipGetErrorString(e));
  return ok();
}

hines_status hines_plan_info_get(const hines_plan* p, hines_plan_info* info) {
  if (!p || !info) return set_err(HINES_ERR_NULL, "NULL argument");
  std::memset(info, 0, sizeof *info);
  info->n = p->host.n;
  info->ncells = p->host.ncells;
  info->nbranches = p->host.nbranches;
  info->ngroups = p->host.ngroups;
  info->nsegments = p->host.nseg;
  info->max_level = p->host.max_level;
  int nb = 0;
  for (const auto& b : p->buckets) nb += b.count > 0;
  info->nclasses = nb;
  info->device_table_bytes = p->dev_bytes;
  info->max_group_lds_bytes = p->max_lds;
  info->kernel = p->host.scheduled ? 1 : (p->host.opt.bitwise ? 2 : 0);
  int32_t mk = 0;
  if (p->host.scheduled)
    for (const auto& G : p->host.kgroup) mk = std::max(mk, G.makespan);
  info->max_makespan = mk;
  return ok();
}

hines_status hines_get_table(const hines_plan* p, int32_t which, int64_t* host_out, int64_t capacity, int64_t* count) {
  if (!p || !count) return set_err(HINES_ERR_NULL, "NULL argument");
  int64_t c = hines::export_table(p->host, which, nullptr, 0);
  if (c < 0) return set_err(HINES_ERR_OPTION, "unknown table %d or tables not kept", which);
  *count = c;
  if (host_out) {
    if (capacity < c) return set_err(HINES_ERR_OPTION, "capacity %lld < %lld", (long long)capacity, (long long)c);
    hines::export_table(p->host, which, host_out, capacity);
  }
  return ok();
}

hines_status hines_destroy(hines_plan* p) {
  if (!p) return ok();
  hines_status st = HINES_OK;
  if (p->dev_mem) {
    int prev = -1;
    hipGetDevice(&prev);
    if (prev != p->device) hipSetDevice(p->device);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipFree(p->dev_mem);
    if (e != hipSuccess) st = set_err(HINES_ERR_HIP, "destroy: %s", hipGetErrorString(e));
    if (prev != p->device && prev >= 0) hipSetDevice(prev);
  }
  delete p;
  return st == HINES_OK ? ok() : st;
}

const char* hines_status_str(hines_status s) {
  switch (s) {
    case HINES_OK: return "ok";
    case HINES_ERR_NULL: return "null pointer";
    case HINES_ERR_BAD_OFFSETS: return "bad cell offsets";
    case HINES_ERR_BAD_PARENT: return "bad parent array";
    case HINES_ERR_BAD_BRANCHES: return "bad branch layout";
    case HINES_ERR_TOO_WIDE: return "level too wide";
    case HINES_ERR_NCELLS: return "cell count mismatch";
    case HINES_ERR_OPTION: return "bad option";
    case HINES_ERR_OOM: return "out of memory";
    case HINES_ERR_HIP: return "HIP error";
    case HINES_ERR_TOO_BIG: return "group too big for LDS";
    case HINES_ERR_NOT_SDD: return "matrix not strictly diagonally dominant";
    case HINES_ERR_STATE: return "invalid state";
  }
  return "unknown status";
}

const char* hines_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
