// MI355X (gfx950) batched Hines solver: plan runtime and the C-ABI declared
// in include/hines.h.  Device code: kernels.hpp.
//
// Design (paper §3-§5 re-thought for CDNA4):
//  * one workgroup solves one packed group of cells (§3: all work of a matrix
//    stays inside one block, so only block-level synchronisation is needed);
//  * every matrix entry crosses HBM once: a group is staged into LDS,
//    eliminated there and its solution written back (the role of the paper's
//    interleaved layout, §5, is played by the LDS image); groups too large
//    for LDS run the level-synchronous sweeps on a global workspace image;
//  * fast path (flow kernel): one wave per group runs a static step schedule
//    built by the setup: in each step every busy lane eliminates one
//    compartment, heavy children hand their contribution to the parent in
//    registers, light children add theirs into the parent's LDS entry, and
//    the compartments of a step sit in consecutive LDS entries, so a step's
//    LDS traffic is conflict-free and needs no per-lane bookkeeping;
//  * level-synchronous path (§3, §4 Fig 4.1): one lane per branch, lanes of
//    a level sorted by branch length, a barrier between levels; children
//    store their contribution in their own slot and the parent pulls them in
//    a fixed order (used for re-rooted plans, bitwise mode and workspace
//    groups);
//  * groups are bucketed by LDS footprint, one launch per bucket, so the
//    occupancy follows the footprint; inside a launch the groups with the
//    longest critical path come first.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/hines.h"
#include "kernels.hpp"
#include "setup.hpp"

// Scratch of hines_solve_noalloc: the (f, y) factors of the cell-lane solve,
// 16 bytes per walk slot, in a file-scope device array instead of the plan's
// allocation.  Each device holds its own copy for the life of the process.  In
// host code the name `scratch` is not a device address: its address on a
// device comes from hipGetSymbolAddress (static_scratch_init), taken once per
// device with the device current, and only that address is passed to kernels.
constexpr int64_t kStaticScratchBytes = (int64_t)256 << 20;
static __device__ __align__(256) double scratch[kStaticScratchBytes / 8];

using hdev::DevTables;
using hdev::RhsSpec;
using hines::KBranch;
using hines::KCell;
using hines::KGroup;
using hines::LdsLayout;

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

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

// Resolve `scratch` on device dev (the current device), once per device.
hipError_t static_scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess) g_scratch_ptr[dev] = ptr;
  return e;
}

void* static_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[dev];
}

// LDS footprint classes (bytes); a launch reserves its class's size per
// workgroup.  A CU holds floor(160 KiB / size) such workgroups, so the classes
// sit at 160 KiB / n (rounded down to 256 bytes) for the occupancies that
// matter; each class is one launch, so there are few of them.
constexpr int kBuckets[] = {4096, 8192, 12288, 16384, 20480, 23296, 27136, 32768, 40960, 54528, 81920, 163840};
constexpr int kGlobalT = 256;  // workgroup of groups whose image lives in the workspace

inline LdsLayout layout_of(const KGroup& g) {
  return LdsLayout{g.ws_off >= 0 ? 0 : g.nunk, (g.nbr + 1) & ~1, g.nlev};
}

}  // namespace

struct hines_plan {
  hines::HostPlan host;
  int device = -1;
  void* dev_mem = nullptr;
  void* scr_mem = nullptr;  // cell-lane kernel: (f, y) scratch
  int64_t dev_bytes = 0;    // dev_mem and scr_mem together
  int64_t scr_bytes = 0;
  DevTables t{};
  struct Bucket {
    int32_t lds_bytes, first, count, global;
    int32_t level;  // 1: level-synchronous kernel for an LDS group of a flow plan
  };
  std::vector<Bucket> buckets;
  std::vector<Bucket> mixed_buckets;  // FP32+refinement kernel (its own LDS layout)
  std::vector<Bucket> res_buckets;    // LDS-resident kernel, by LDS class
  // LDS classes launch concurrently: bucket i runs on res_lane[i] (0: the
  // caller's stream, k > 0: res_streams[k - 1]), forked from and joined back
  // into the caller's stream with events, so groups of different classes
  // share CUs and no class waits for the tail of another
  static constexpr int kResStreams = 3;
  hipStream_t res_streams[kResStreams] = {};
  hipEvent_t res_fork = nullptr;
  hipEvent_t res_join[kResStreams] = {};
  std::vector<int32_t> res_lane;
  ~hines_plan() {
    for (int k = 0; k < kResStreams; ++k) {
      if (res_streams[k]) (void)hipStreamDestroy(res_streams[k]);
      if (res_join[k]) (void)hipEventDestroy(res_join[k]);
    }
    if (res_fork) (void)hipEventDestroy(res_fork);
  }
  std::vector<int32_t> res_list;      // resident group ids in launch order
  bool mixed_ok = false;              // every group fits the mixed layout in LDS
  int64_t max_lds = 0;
  // user-numbering tables of the element-wise kernels, uploaded on first use
  std::vector<int32_t> parent_host;
  std::vector<int64_t> cell_off_host;
  void* adj_mem = nullptr;
  int64_t adj_bytes = 0;
  const int32_t* d_parent = nullptr;
  const int32_t* d_ch_off = nullptr;
  const int32_t* d_ch = nullptr;
  const int64_t* d_cell_off = nullptr;
  unsigned long long* d_flag = nullptr;  // result word of hines_check_matrix
};

struct hines_timeloop {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int32_t nsteps = 0;
  void* mem = nullptr;  // cell-lane plans: factors and walk-layout arrays of the loop
  int64_t bytes = 0;
};

namespace {

// Device bytes the library holds, and a cap on them: HINES_DEVICE_BYTE_CAP
// (unset: no cap).  A request past the cap fails as if the device were full,
// so that the out-of-memory paths can be exercised on any GPU.
std::atomic<int64_t> g_dev_bytes{0};

int64_t device_byte_cap() {
  static const int64_t cap = [] {
    const char* e = std::getenv("HINES_DEVICE_BYTE_CAP");
    return e ? std::atoll(e) : (int64_t)-1;
  }();
  return cap;
}

hipError_t dev_alloc(void** ptr, int64_t bytes) {
  const int64_t cap = device_byte_cap();
  if (cap >= 0 && g_dev_bytes.load() + bytes > cap) {
    *ptr = nullptr;
    return hipErrorOutOfMemory;
  }
  const hipError_t e = hipMalloc(ptr, (size_t)bytes);
  if (e == hipSuccess) g_dev_bytes += bytes;
  return e;
}

hipError_t dev_free(void* ptr, int64_t bytes) {
  const hipError_t e = hipFree(ptr);
  if (e == hipSuccess) g_dev_bytes -= bytes;
  return e;
}

template <int T, int MODE>
void launch_level(const DevTables& t, const hines_plan::Bucket& bk, const RhsSpec& rs, const double* d,
                  const double* u, double* x, hipStream_t s) {
  if (bk.global)
    hipLaunchKernelGGL((hdev::k_solve_level<kGlobalT, MODE, true>), dim3(bk.count), dim3(kGlobalT), bk.lds_bytes, s,
                       t, rs, d, u, x);
  else
    hipLaunchKernelGGL((hdev::k_solve_level<T, MODE, false>), dim3(bk.count), dim3(T), bk.lds_bytes, s, t, rs, d,
                       u, x);
}

template <int T>
void launch_bucket(const hines_plan* p, const hines_plan::Bucket& bk, const RhsSpec& rs, const double* d,
                   const double* u, double* x, hipStream_t s) {
  DevTables t = p->t;
  t.glist = p->t.glist + bk.first;
  if (p->host.flow && !bk.global && !bk.level) {
    if (rs.mode == hdev::kRhsGiven)
      hipLaunchKernelGGL(hdev::k_solve_flow<hdev::kFlowGiven>, dim3(bk.count), dim3(64), bk.lds_bytes, s, t, rs, d, u, x);
    else if (rs.mode == hdev::kRhsNoise)
      hipLaunchKernelGGL(hdev::k_solve_flow<hdev::kFlowNoise>, dim3(bk.count), dim3(64), bk.lds_bytes, s, t, rs, d, u, x);
    else if (rs.icur)
      hipLaunchKernelGGL(hdev::k_solve_flow<hdev::kFlowCVI>, dim3(bk.count), dim3(64), bk.lds_bytes, s, t, rs, d, u, x);
    else
      hipLaunchKernelGGL(hdev::k_solve_flow<hdev::kFlowCV>, dim3(bk.count), dim3(64), bk.lds_bytes, s, t, rs, d, u, x);
  } else if (p->host.opt.bitwise) {
    launch_level<T, hdev::kModeBitwise>(t, bk, rs, d, u, x, s);
  } else if (p->host.all_ascending) {
    launch_level<T, hdev::kModeAscending>(t, bk, rs, d, u, x, s);
  } else {
    launch_level<T, hdev::kModeFast>(t, bk, rs, d, u, x, s);
  }
}

// one instantiation of the resident kernel per LDS class (plane stride S)
template <int C>
void launch_res_class(const DevTables& t, int32_t count, const double* d, const double* u, const double* b, double* x,
                      hipStream_t s) {
  hipLaunchKernelGGL(hdev::k_solve_res<hines::kResClassStride[C]>, dim3((unsigned)count), dim3(64),
                     hines::kResClassBytes[C], s, t, d, u, b, x);
}

template <int C = 0>
hipError_t res_class_attr() {
  if constexpr (C < hines::kResClasses) {
    hipError_t e = hipFuncSetAttribute((const void*)hdev::k_solve_res<hines::kResClassStride[C]>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, hines::kResClassBytes[C]);
    return e == hipSuccess ? res_class_attr<C + 1>() : e;
  } else {
    return hipSuccess;
  }
}

template <int C = 0>
void launch_res(int32_t cls, const DevTables& t, int32_t count, const double* d, const double* u, const double* b,
                double* x, hipStream_t s) {
  if constexpr (C < hines::kResClasses) {
    if (cls == C)
      launch_res_class<C>(t, count, d, u, b, x, s);
    else
      launch_res<C + 1>(cls, t, count, d, u, b, x, s);
  }
}

hipError_t launch_resident(const hines_plan* p, const double* d, const double* u, const double* b, double* x,
                           hipStream_t s) {
  bool used[hines_plan::kResStreams] = {};
  for (size_t i = 0; i < p->res_buckets.size(); ++i)
    if (p->res_lane[i] > 0) used[p->res_lane[i] - 1] = true;
  hipError_t e = hipSuccess;
  bool fork = false;
  for (int k = 0; k < hines_plan::kResStreams; ++k) fork = fork || used[k];
  if (fork) {
    e = hipEventRecord(p->res_fork, s);
    for (int k = 0; k < hines_plan::kResStreams && e == hipSuccess; ++k)
      if (used[k]) e = hipStreamWaitEvent(p->res_streams[k], p->res_fork, 0);
    if (e != hipSuccess) return e;
  }
  for (size_t i = 0; i < p->res_buckets.size(); ++i) {
    const auto& bk = p->res_buckets[i];
    DevTables t = p->t;
    t.rlist = p->t.rlist + bk.first;
    const hipStream_t si = p->res_lane[i] > 0 ? p->res_streams[p->res_lane[i] - 1] : s;
    launch_res(bk.level, t, bk.count, d, u, b, x, si);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  for (int k = 0; k < hines_plan::kResStreams && e == hipSuccess; ++k)
    if (used[k]) {
      e = hipEventRecord(p->res_join[k], p->res_streams[k]);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, p->res_join[k], 0);
    }
  return e;
}

hipError_t launch_solve(const hines_plan* p, const RhsSpec& rs, const double* d, const double* u, double* x,
                        hipStream_t s) {
  if (p->host.res.built && rs.mode == hdev::kRhsGiven) return launch_resident(p, d, u, rs.rhs, x, s);
  if (p->host.sq.built) {
    const dim3 grid((unsigned)p->host.sq.nwaves);
    if (rs.mode == hdev::kRhsGiven)
      hipLaunchKernelGGL(hdev::k_solve_seq<hdev::kFlowGiven>, grid, dim3(64), 0, s, p->t, rs, d, u, x);
    else if (rs.mode == hdev::kRhsNoise)
      hipLaunchKernelGGL(hdev::k_solve_seq<hdev::kFlowNoise>, grid, dim3(64), 0, s, p->t, rs, d, u, x);
    else if (rs.icur)
      hipLaunchKernelGGL(hdev::k_solve_seq<hdev::kFlowCVI>, grid, dim3(64), 0, s, p->t, rs, d, u, x);
    else
      hipLaunchKernelGGL(hdev::k_solve_seq<hdev::kFlowCV>, grid, dim3(64), 0, s, p->t, rs, d, u, x);
    return hipGetLastError();
  }
  if (p->host.cl.built) {
    const dim3 grid((unsigned)p->host.cl.nwaves);
    if (rs.mode == hdev::kRhsGiven)
      hipLaunchKernelGGL(hdev::k_solve_cells<hdev::kFlowGiven>, grid, dim3(64), 0, s, p->t, rs, d, u, x);
    else if (rs.mode == hdev::kRhsNoise)
      hipLaunchKernelGGL(hdev::k_solve_cells<hdev::kFlowNoise>, grid, dim3(64), 0, s, p->t, rs, d, u, x);
    else if (rs.icur)
      hipLaunchKernelGGL(hdev::k_solve_cells<hdev::kFlowCVI>, grid, dim3(64), 0, s, p->t, rs, d, u, x);
    else
      hipLaunchKernelGGL(hdev::k_solve_cells<hdev::kFlowCV>, grid, dim3(64), 0, s, p->t, rs, d, u, x);
    return hipGetLastError();
  }
  for (const auto& bk : p->buckets) {
    if (bk.count == 0) continue;
    switch (p->host.opt.group_width) {
      case 64: launch_bucket<64>(p, bk, rs, d, u, x, s); break;
      case 128: launch_bucket<128>(p, bk, rs, d, u, x, s); break;
      case 256: launch_bucket<256>(p, bk, rs, d, u, x, s); break;
      case 512: launch_bucket<512>(p, bk, rs, d, u, x, s); break;
      default: launch_bucket<1024>(p, bk, rs, d, u, x, s); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_mixed(const hines_plan* p, const float* d32, const float* u32, const double* b, double* x,
                        int sweeps, hipStream_t s) {
  for (const auto& bk : p->mixed_buckets) {
    if (bk.count == 0) continue;
    DevTables t = p->t;
    t.glist = p->t.glist + bk.first;
    switch (p->host.opt.group_width) {
      case 64: hipLaunchKernelGGL(hdev::k_solve_mixed<64>, dim3(bk.count), dim3(64), bk.lds_bytes, s, t, d32, u32, b, x, sweeps); break;
      case 128: hipLaunchKernelGGL(hdev::k_solve_mixed<128>, dim3(bk.count), dim3(128), bk.lds_bytes, s, t, d32, u32, b, x, sweeps); break;
      case 256: hipLaunchKernelGGL(hdev::k_solve_mixed<256>, dim3(bk.count), dim3(256), bk.lds_bytes, s, t, d32, u32, b, x, sweeps); break;
      case 512: hipLaunchKernelGGL(hdev::k_solve_mixed<512>, dim3(bk.count), dim3(512), bk.lds_bytes, s, t, d32, u32, b, x, sweeps); break;
      default: hipLaunchKernelGGL(hdev::k_solve_mixed<1024>, dim3(bk.count), dim3(1024), bk.lds_bytes, s, t, d32, u32, b, x, sweeps); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int T>
hipError_t allow_lds_t() {
  const void* fns[] = {(const void*)hdev::k_solve_level<T, hdev::kModeFast, false>,
                       (const void*)hdev::k_solve_level<T, hdev::kModeBitwise, false>,
                       (const void*)hdev::k_solve_level<T, hdev::kModeAscending, false>,
                       (const void*)hdev::k_solve_mixed<T>};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)hines::kLdsLimitBytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t allow_lds(int T) {
  const void* fns[] = {(const void*)hdev::k_solve_flow<hdev::kFlowGiven>,
                       (const void*)hdev::k_solve_flow<hdev::kFlowCV>,
                       (const void*)hdev::k_solve_flow<hdev::kFlowCVI>,
                       (const void*)hdev::k_solve_flow<hdev::kFlowNoise>,
                       (const void*)hdev::k_solve_level<kGlobalT, hdev::kModeFast, true>,
                       (const void*)hdev::k_solve_level<kGlobalT, hdev::kModeBitwise, true>,
                       (const void*)hdev::k_solve_level<kGlobalT, hdev::kModeAscending, true>};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)hines::kLdsLimitBytes);
    if (e != hipSuccess) return e;
  }
  switch (T) {
    case 64: return allow_lds_t<64>();
    case 128: return allow_lds_t<128>();
    case 256: return allow_lds_t<256>();
    case 512: return allow_lds_t<512>();
    case 1024: return allow_lds_t<1024>();
  }
  return hipErrorInvalidValue;
}

// Every index a kernel derives from the tables must stay inside the group's
// image; checked once on the host before anything is uploaded.  The static
// schedule is checked for its ordering invariants as well.
bool check_kernel_tables(const hines::HostPlan& P, std::string& why, bool& capacity) {
  capacity = false;
  if (!P.kernel_tables_fit) {
    why = "a group exceeds the int16 branch records";
    capacity = true;
    return false;
  }
  const int64_t pad = hines::kLdsPad;
  for (int64_t g = 0; g < P.ngroups; ++g) {
    const KGroup& G = P.kgroup[g];
    if (G.seg_begin < 0 || G.seg_begin + G.nlev + 1 > (int64_t)P.kseg.size() || G.br_begin != P.kseg[G.seg_begin] ||
        P.kseg[G.seg_begin + G.nlev] - G.br_begin != G.nbr || G.nlev < 1) {
      why = "segment range";
      return false;
    }
    if (layout_of(G).bytes() > hines::kLdsLimitBytes) {
      why = "the branch tables of a group exceed LDS";
      capacity = true;
      return false;
    }
    if (G.ws_off >= 0 && G.ws_off + 3 * (int64_t)G.nunk > P.ws_doubles) {
      why = "workspace range";
      return false;
    }
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
    for (int e = G.br_begin; e < G.br_begin + G.nbr; ++e) {
      const KBranch& B = P.kbranch[e];
      const int len = B.lendir > 0 ? B.lendir : -B.lendir;
      const int dir = B.lendir > 0 ? 1 : -1;
      const int last = B.start + dir * (len - 1);
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
  if (P.flow) {
    // every LDS index the flow kernel forms: entries R + j c + rank < nent,
    // push ranks < naux, stored entries and push targets < nent
    if ((int64_t)P.kflow.size() != P.ngroups) {
      why = "flow table size";
      return false;
    }
    std::vector<uint8_t> seen;
    for (int64_t g = 0; g < P.ngroups; ++g) {
      const KGroup& G = P.kgroup[g];
      const hines::KFlow& W = P.kflow[g];
      if (G.ws_off >= 0) continue;
      if (W.nstep == 0 && W.nelem == 0 && W.naux == 0) continue;  // level kernel in LDS
      if (W.nstep < 1 || W.nstep > hines::kMaxSteps || W.nelem != G.user_n || W.naux < 0 || W.nent < W.nelem ||
          hines::flow_image8(W) > 32767 || W.nent % hines::kFlowChunk || W.step_off < 0 || 2 * (W.step_off + W.nstep) > (int64_t)P.fmask.size() ||
          W.pos_off < 0 || W.pos_off + W.nelem > (int64_t)P.fpos.size() || W.aux_off < 0 || (W.aux_off & 1) ||
          W.aux_off + W.naux + 1 > (int64_t)P.faux.size() + 1 || hines::flow_lds_bytes(W) > hines::kLdsLimitBytes) {
        why = "flow group record";
        capacity = hines::flow_lds_bytes(W) > hines::kLdsLimitBytes;
        return false;
      }
      int64_t act = 0, push = 0;
      for (int32_t t = 0; t < W.nstep; ++t) {
        const uint64_t M = P.fmask[2 * (W.step_off + t)], E = P.fmask[2 * (W.step_off + t) + 1];
        if (E & ~M) {
          why = "flow push outside the active lanes";
          return false;
        }
        act += __builtin_popcountll(M);
        push += __builtin_popcountll(E);
      }
      if (act * hines::kFlowChunk != W.nent || push != W.naux) {
        why = "flow mask counts";
        return false;
      }
      const int32_t nunits = W.nent / hines::kFlowChunk * hines::kFlowBlock8;  // block region
      auto valid = [&](int32_t q) {
        const int32_t r = q % hines::kFlowBlock8;
        return q >= 0 && q < nunits && r < 3 * hines::kFlowChunk && r % 3 == 0;
      };
      seen.assign(nunits, 0);
      for (int32_t e = 0; e < W.nelem; ++e) {
        const int32_t q = P.fpos[W.pos_off + e] & 0x7fff;
        if (!valid(q) || seen[q]) {
          why = "flow positions";
          return false;
        }
        seen[q] = 1;
      }
      for (int32_t k = 0; k < W.naux; ++k) {
        if (!valid(P.faux[W.aux_off + k])) {
          why = "flow push target";
          return false;
        }
      }
    }
  }
  return true;
}

// Cell-lane tables: every wave's chunks inside the tables, every position
// inside its lane's cell, and per lane a stack that never underflows nor
// leaves its kCellStack LDS slots, in both sweeps, so that no kernel access
// leaves its buffers whatever the tables hold.
bool check_cell_tables(const hines::HostPlan& P, const int64_t* cell_offsets, std::string& why) {
  const hines::CellLanes& C = P.cl;
  if ((int64_t)C.range.size() != 64 * C.nwaves || (int64_t)C.mbsrc.size() != 64 * C.nwaves) {
    why = "per-lane tables of the wrong size";
    return false;
  }
  for (int64_t w = 0; w < C.nwaves; ++w) {
    const hines::KCellWave& W = C.waves[w];
    if (W.chunk_off < 0 || W.nchunk < 0 || W.chunk_off + W.nchunk > C.nchunks || W.ncell < 1 || W.ncell > 64) {
      why = "wave " + std::to_string(w) + " record out of range";
      return false;
    }
    for (int c = 0; c < 64; ++c) {
      const int32_t cell = C.lane_cell[w * 64 + c];
      const int64_t lo = C.base[w * 64 + c];
      int64_t size = 0;
      if (cell >= 0) {
        if (cell >= P.ncells || lo != cell_offsets[cell]) {
          why = "wave " + std::to_string(w) + " lane cell out of range";
          return false;
        }
        size = cell_offsets[cell + 1] - lo;
      } else if (lo != 0) {
        why = "empty lane with a base";
        return false;
      }
      // the steps outside the lane's range are its padding, and only those
      // (the step kernel reads the zero block in their place)
      const uint64_t rg = C.range[w * 64 + c];
      const int64_t q0 = (int64_t)(rg & 0xffffffffu), q1 = (int64_t)(rg >> 32);
      if (q0 > q1 || q1 > (int64_t)W.nchunk * hines::kCellChunk || (cell < 0 && rg != 0)) {
        why = "wave " + std::to_string(w) + " lane " + std::to_string(c) + " step range out of bounds";
        return false;
      }
      // stack entries per sweep (the top in registers, the rest in slots 1..)
      int m = 0;
      bool ok_b = true;
      for (int64_t k = 0; k < W.nchunk && ok_b; ++k)
        for (int e = 0; e < hines::kCellChunk && ok_b; ++e) {
          const int64_t g = W.chunk_off + k;
          const uint8_t f = C.flags[hines::cell_flag_index(g, c, e)];
          const uint16_t ps = C.pos[hines::cell_pos_index(g, c, e)];
          if ((ps == hines::kCellPadPos) != ((f & hines::CF_PAD) != 0) || (ps != hines::kCellPadPos && ps >= size)) {
            why = "wave " + std::to_string(w) + " position out of range";
            return false;
          }
          const int64_t q = k * hines::kCellChunk + e;
          if (((f & hines::CF_PAD) != 0) == (q >= q0 && q < q1)) {
            why = "wave " + std::to_string(w) + " lane " + std::to_string(c) + " padding outside its step range";
            return false;
          }
          if (f & hines::CF_POP) ok_b = m-- >= 1;
          if ((f & hines::CF_MERGE) && m < 1) ok_b = false;
          if (f & hines::CF_PUSH) ok_b = ok_b && m++ < hines::kCellStack;
        }
      if (!ok_b || m != 0) {
        why = "wave " + std::to_string(w) + " lane " + std::to_string(c) + " backward stack unbalanced";
        return false;
      }
      bool ok_f = true;
      for (int64_t k = W.nchunk - 1; k >= 0 && ok_f; --k)
        for (int e = hines::kCellChunk - 1; e >= 0 && ok_f; --e) {
          const uint8_t f = C.flags[hines::cell_flag_index(W.chunk_off + k, c, e)];
          if ((f & (hines::CF_PUSH | hines::CF_MERGE)) && m < 1) ok_f = false;
          if (f & hines::CF_PUSH) --m;
          if (f & hines::CF_POP) ok_f = ok_f && m++ < hines::kCellStack;
        }
      if (!ok_f || m != 0) {
        why = "wave " + std::to_string(w) + " lane " + std::to_string(c) + " forward stack unbalanced";
        return false;
      }
    }
    // mailboxes: a lane posts at most once (the root of its cut-off subtree);
    // every post is taken exactly once, by a lane of the same cell, at a
    // strictly later step, from the mailbox its source list names next; the
    // forward list is the backward list reversed
    const int64_t steps = (int64_t)W.nchunk * hines::kCellChunk;
    int64_t post_at[64];
    int taken[64] = {0};
    for (int c = 0; c < 64; ++c) {
      post_at[c] = -1;
      int no = 0;
      for (int64_t q = 0; q < steps; ++q) {
        const uint8_t f = C.flags[hines::cell_flag_index(W.chunk_off + q / hines::kCellChunk, c, (int)(q % hines::kCellChunk))];
        if (f & hines::CF_MBOUT) {
          ++no;
          post_at[c] = q;
        }
      }
      if (no > 1) {
        why = "wave " + std::to_string(w) + " lane " + std::to_string(c) + " posts more than once";
        return false;
      }
    }
    for (int c = 0; c < 64; ++c) {
      const uint64_t ms = C.mbsrc[w * 64 + c];
      const uint32_t bw = (uint32_t)ms, fw = (uint32_t)(ms >> 32);
      int src[6], ni = 0;
      bool ok = true;
      for (int64_t q = 0; q < steps && ok; ++q) {
        const uint8_t f = C.flags[hines::cell_flag_index(W.chunk_off + q / hines::kCellChunk, c, (int)(q % hines::kCellChunk))];
        if (!(f & hines::CF_MBIN)) continue;
        if (ni >= 5) {
          ok = false;
          break;
        }
        const int s = (int)((bw >> (6 * ni)) & 63u);
        src[ni++] = s;
        ok = s != c && post_at[s] >= 0 && post_at[s] < q && C.lane_cell[w * 64 + s] == C.lane_cell[w * 64 + c] &&
             taken[s]++ == 0;
      }
      uint32_t bw2 = 0, fw2 = 0;
      for (int i = 0; i < ni && ok; ++i) {
        bw2 |= (uint32_t)src[i] << (6 * i);
        fw2 |= (uint32_t)src[ni - 1 - i] << (6 * i);
      }
      if (!ok || bw != bw2 || fw != fw2) {
        why = "wave " + std::to_string(w) + " lane " + std::to_string(c) + " mailbox takes unpaired or out of order";
        return false;
      }
    }
    for (int c = 0; c < 64; ++c)
      if ((post_at[c] >= 0) != (taken[c] == 1)) {
        why = "wave " + std::to_string(w) + " lane " + std::to_string(c) + " mailbox post not taken";
        return false;
      }
  }
  return true;
}

hines_status check_call(const hines_plan* p, int32_t ncells) {
  if (!p) return set_err(HINES_ERR_NULL, "plan is NULL");
  if (p->host.opt.host_only) return set_err(HINES_ERR_STATE, "plan was built host_only");
  if (ncells != p->host.ncells)
    return set_err(HINES_ERR_NCELLS, "ncells %d != plan's %lld", ncells, (long long)p->host.ncells);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return set_err(HINES_ERR_STATE, "current device %d is not the plan's device %d", dev, p->device);
  return HINES_OK;
}

hines_status run_solve(const hines_plan* p, const RhsSpec& rs, const double* diag, const double* upper, double* x,
                       void* stream) {
  hipError_t e = launch_solve(p, rs, diag, upper, x, (hipStream_t)stream);
  if (e != hipSuccess) return set_err(HINES_ERR_HIP, "launch: %s", hipGetErrorString(e));
  return ok();
}

// Children lists (CSR, ascending child index), parent array and cell offsets
// on the device, for the element-wise kernels.
hines_status ensure_adjoint_tables(hines_plan* p) {
  if (p->adj_mem) return HINES_OK;
  const int64_t n = p->host.n;
  const std::vector<int32_t>& par = p->parent_host;
  std::vector<int32_t> off(n + 1, 0), ch(n > 0 ? n : 1, 0);
  for (int64_t i = 0; i < n; ++i)
    if (par[i] >= 0) ++off[par[i] + 1];
  for (int64_t i = 0; i < n; ++i) off[i + 1] += off[i];
  std::vector<int32_t> fill(off.begin(), off.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    if (par[i] >= 0) ch[fill[par[i]]++] = (int32_t)i;
  auto al = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
  const int64_t sp = al(4 * std::max<int64_t>(n, 1)), so = al(4 * (n + 1)), sc = al(4 * std::max<int64_t>(n, 1)),
                sf = al(8 * (int64_t)p->cell_off_host.size());
  void* mem = nullptr;
  const int64_t bytes = sp + so + sc + sf + 256;
  hipError_t e = dev_alloc(&mem, bytes);
  if (e != hipSuccess) return set_err(HINES_ERR_OOM, "element-wise tables: %s", hipGetErrorString(e));
  char* b = (char*)mem;
  if (n > 0) e = hipMemcpy(b, par.data(), 4 * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b + sp, off.data(), 4 * (n + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess && n > 0) e = hipMemcpy(b + sp + so, ch.data(), 4 * n, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b + sp + so + sc, p->cell_off_host.data(), 8 * p->cell_off_host.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    dev_free(mem, bytes);
    return set_err(HINES_ERR_HIP, "element-wise table upload: %s", hipGetErrorString(e));
  }
  p->adj_mem = mem;
  p->adj_bytes = bytes;
  p->d_parent = (const int32_t*)b;
  p->d_ch_off = (const int32_t*)(b + sp);
  p->d_ch = (const int32_t*)(b + sp + so);
  p->d_cell_off = (const int64_t*)(b + sp + so + sc);
  p->d_flag = (unsigned long long*)(b + sp + so + sc + sf);
  return HINES_OK;
}

inline dim3 grid_for(int64_t n, int block) { return dim3((unsigned)((n + block - 1) / block)); }

hines_status launched() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(HINES_ERR_HIP, "launch: %s", hipGetErrorString(e));
  return ok();
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
  opt->max_group_unknowns = 1536;
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
  if (opt.reserved[0] != 0) return set_err(HINES_ERR_OPTION, "reserved option fields must be 0");
  if (opt.cell_cut_percent < 0 || opt.cell_max_cuts < 0 || opt.cell_max_cuts > hines::kCellMaxCuts ||
      opt.res_pack < 0 || opt.res_pack > hines::kResMaxSlots)
    return set_err(HINES_ERR_OPTION, "tuning option out of range");
  if (opt.cell_lanes < 0 || opt.cell_lanes > 2) return set_err(HINES_ERR_OPTION, "cell_lanes must be 0, 1 or 2");
  if (opt.cell_lanes && opt.bitwise)
    return set_err(HINES_ERR_OPTION, "cell_lanes needs the fast arithmetic form (bitwise 0)");
  if (opt.resident && (opt.bitwise || opt.cell_lanes))
    return set_err(HINES_ERR_OPTION, "resident needs bitwise 0 and cell_lanes 0");
  hines::Options o;
  o.rebalance_root = opt.rebalance_root != 0;
  o.split_branches = opt.split_branches;
  o.level_balance = opt.level_balance;
  o.group_width = opt.group_width;
  o.cell_order = opt.cell_order;
  o.max_group_unknowns = opt.max_group_unknowns;
  o.host_only = opt.host_only != 0;
  o.keep_tables = opt.keep_tables != 0;
  o.bitwise = opt.bitwise != 0;
  o.scheduler = opt.level_sync ? 0 : 1;
  o.cell_lanes = opt.cell_lanes == 1;
  o.cell_seq = opt.cell_lanes == 2;
  o.resident = opt.resident != 0;
  if (opt.cell_cut_percent > 0) o.cell_cut_percent = opt.cell_cut_percent;
  if (opt.cell_max_cuts > 0) o.cell_max_cuts = opt.cell_max_cuts;
  if (opt.res_pack > 0) o.res_pack = opt.res_pack;
  if (o.cell_lanes || o.cell_seq) o.scheduler = 0;  // the groups serve the other forms only
  hines_plan* p = new (std::nothrow) hines_plan();
  if (!p) return set_err(HINES_ERR_OOM, "host allocation failed");
  std::string why;
  // the host tables can take tens of GB for the largest networks: running
  // out of host memory is a status, not an exception through the C ABI
  try {
    hines::Status s = hines::build_plan(parent, n, branch_offsets, nbranches, cell_offsets, ncells, o, p->host, why);
    if (s != hines::OK) {
      delete p;
      return set_err((hines_status)s, "%s", why.c_str());
    }
    if (o.cell_lanes) {
      s = hines::build_cell_lanes(parent, n, cell_offsets, ncells, p->host.cl, why, o.cell_cut_percent,
                                  o.cell_max_cuts);
      if (s == hines::OK && !check_cell_tables(p->host, cell_offsets, why)) s = hines::ERR_STATE;
      if (s != hines::OK) {
        delete p;
        return set_err((hines_status)s, "cell lanes: %s", why.c_str());
      }
    }
    if (o.cell_seq) {
      s = hines::build_seq_lanes(parent, n, cell_offsets, ncells, p->host.sq, why, o.cell_cut_percent,
                                 o.cell_max_cuts);
      if (s == hines::OK && !hines::check_seq_lanes(p->host.sq, parent, n, cell_offsets, ncells, why))
        s = hines::ERR_STATE;
      if (s != hines::OK) {
        delete p;
        return set_err((hines_status)s, "index-order cell lanes: %s", why.c_str());
      }
    }
    if (o.resident) {
      s = hines::build_resident(parent, n, cell_offsets, ncells, p->host.res, why, o.res_pack, o.rebalance_root);
      if (s == hines::OK && !hines::check_resident(p->host.res, parent, n, why)) s = hines::ERR_STATE;
      if (s != hines::OK) {
        delete p;
        return set_err((hines_status)s, "resident: %s", why.c_str());
      }
    }
  } catch (const std::bad_alloc&) {
    delete p;
    return set_err(HINES_ERR_OOM, "host memory exhausted while building the plan tables");
  }
  bool capacity = false;
  bool groups_usable = true;
  if (!o.host_only && !check_kernel_tables(p->host, why, capacity)) {
    if ((o.cell_lanes || o.cell_seq) && capacity) {
      // the cell-lane kernels never read the group tables; only the groups'
      // FP32+refinement solve needs them, and it is refused on this plan
      groups_usable = false;
    } else {
      delete p;
      return set_err(capacity ? HINES_ERR_TOO_BIG : HINES_ERR_STATE, "kernel tables: %s", why.c_str());
    }
  }
  const hines::HostPlan& P = p->host;
  // buckets by LDS footprint and kernel: flow groups, level-synchronous LDS
  // groups (plans without a flow schedule, or groups whose schedule does not
  // fit LDS), and groups whose image lives in the workspace
  const int nbk = (int)(sizeof kBuckets / sizeof kBuckets[0]);
  std::vector<std::vector<int32_t>> members(2 * nbk + 1);
  int64_t global_lds = 0;
  for (int64_t g = 0; g < P.ngroups; ++g) {
    const KGroup& G = P.kgroup[g];
    if (G.ws_off >= 0) {
      const int64_t bytes = layout_of(G).bytes();
      p->max_lds = std::max(p->max_lds, bytes);
      members[2 * nbk].push_back((int32_t)g);
      global_lds = std::max(global_lds, bytes);
      continue;
    }
    const bool fl = P.flow && P.kflow[g].nstep > 0;
    const int64_t bytes = fl ? hines::flow_lds_bytes(P.kflow[g]) : layout_of(G).bytes();
    p->max_lds = std::max(p->max_lds, bytes);
    int k = 0;
    while (k < nbk && kBuckets[k] < bytes) ++k;
    if (k == nbk) k = nbk - 1;  // host_only plans only; checked above otherwise
    members[(fl ? 0 : nbk) + k].push_back((int32_t)g);
  }
  std::vector<int32_t> glist;
  for (int k = 0; k <= 2 * nbk; ++k) {
    auto& m = members[k];
    if (m.empty()) continue;
    std::stable_sort(m.begin(), m.end(), [&](int32_t a, int32_t b) { return P.kgroup[a].cost > P.kgroup[b].cost; });
    const bool glob = k == 2 * nbk;
    const int32_t lds = glob ? (int32_t)((global_lds + 255) & ~(int64_t)255) : kBuckets[k % nbk];
    p->buckets.push_back({lds, (int32_t)glist.size(), (int32_t)m.size(), glob ? 1 : 0, (!glob && k >= nbk) ? 1 : 0});
    glist.insert(glist.end(), m.begin(), m.end());
  }
  // buckets of the FP32+refinement kernel (its LDS image holds 32 bytes per slot)
  {
    std::vector<std::vector<int32_t>> mm(nbk);
    p->mixed_ok = groups_usable;
    for (int64_t g = 0; g < P.ngroups && p->mixed_ok; ++g) {
      const int64_t bytes = hdev::mixed_layout(P.kgroup[g]).bytes();
      int k = 0;
      while (k < nbk && kBuckets[k] < bytes) ++k;
      if (k == nbk) p->mixed_ok = false;
      else mm[k].push_back((int32_t)g);
    }
    if (p->mixed_ok)
      for (int k = 0; k < nbk; ++k) {
        auto& m = mm[k];
        std::stable_sort(m.begin(), m.end(), [&](int32_t a, int32_t b) { return P.kgroup[a].cost > P.kgroup[b].cost; });
        p->mixed_buckets.push_back({kBuckets[k], (int32_t)glist.size(), (int32_t)m.size(), 0, 0});
        glist.insert(glist.end(), m.begin(), m.end());
      }
  }
  // resident groups by LDS class, longest schedules first within a class
  if (P.res.built) {
    std::vector<std::vector<int32_t>> rm(hines::kResClasses);
    for (int64_t g = 0; g < (int64_t)P.res.groups.size(); ++g) rm[P.res.groups[g].cls].push_back((int32_t)g);
    for (int k = 0; k < hines::kResClasses; ++k) {
      auto& m = rm[k];
      if (m.empty()) continue;
      std::stable_sort(m.begin(), m.end(), [&](int32_t a, int32_t b) {
        return P.res.groups[a].nchunk > P.res.groups[b].nchunk;
      });
      // Bucket.level carries the LDS class of a resident launch
      p->res_buckets.push_back({hines::kResClassBytes[k], (int32_t)p->res_list.size(), (int32_t)m.size(), 0, k});
      p->res_list.insert(p->res_list.end(), m.begin(), m.end());
    }
    // streams of the class launches: the largest estimated work (chunks of
    // its groups over the groups a CU holds) first, each on the least loaded
    std::vector<double> work(p->res_buckets.size(), 0.0);
    for (size_t i = 0; i < p->res_buckets.size(); ++i) {
      const auto& bk = p->res_buckets[i];
      for (int32_t j = bk.first; j < bk.first + bk.count; ++j) work[i] += P.res.groups[p->res_list[j]].nchunk;
      work[i] /= (double)(hines::kLdsLimitBytes / bk.lds_bytes);
    }
    std::vector<size_t> order(work.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return work[a] > work[b]; });
    double load[hines_plan::kResStreams + 1] = {};
    p->res_lane.assign(p->res_buckets.size(), 0);
    for (size_t i : order) {
      int best = 0;
      for (int k = 1; k <= hines_plan::kResStreams; ++k)
        if (load[k] < load[best]) best = k;
      p->res_lane[i] = best;
      load[best] += work[i];
    }
  }
  if (o.host_only) {
    *out = p;
    return ok();
  }
  p->parent_host.assign(parent, parent + n);
  p->cell_off_host.assign(cell_offsets, cell_offsets + ncells + 1);
  // upload: one allocation, 256-byte aligned sub-buffers
  auto al = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
  const int64_t sz_br = al((int64_t)P.kbranch.size() * sizeof(KBranch));
  const int64_t sz_grp = al((int64_t)P.kgroup.size() * sizeof(KGroup));
  const int64_t sz_seg = al((int64_t)P.kseg.size() * sizeof(int32_t));
  const int64_t sz_cell = al((int64_t)P.kcell.size() * sizeof(KCell));
  const int64_t sz_gl = al((int64_t)glist.size() * sizeof(int32_t));
  const int64_t sz_ws = al(P.ws_doubles * (int64_t)sizeof(double));
  const int64_t sz_fl = al((int64_t)P.kflow.size() * sizeof(hines::KFlow));
  const int64_t sz_fm = al((int64_t)P.fmask.size() * sizeof(uint64_t));
  const int64_t sz_fp = al((int64_t)P.fpos.size() * sizeof(uint16_t));
  const int64_t sz_fa = al((int64_t)P.faux.size() * sizeof(int16_t));
  const hines::CellLanes& CL = P.cl;
  const int64_t sz_cw = al((int64_t)CL.waves.size() * sizeof(hines::KCellWave));
  const int64_t sz_cb = al((int64_t)CL.base.size() * sizeof(int64_t));
  const int64_t sz_cp = al((int64_t)CL.pos.size() * sizeof(uint16_t));
  const int64_t sz_cf = al((int64_t)CL.flags.size());
  const int64_t sz_cm = al((int64_t)CL.mbsrc.size() * sizeof(uint64_t));
  const int64_t sz_cr = al((int64_t)CL.range.size() * sizeof(uint64_t));
  const int64_t sz_cz = CL.built ? al(64 * 16) : 0;  // the step kernel's zero block
  const hines::SeqLanes& SQ = P.sq;
  const int64_t sz_sw = al((int64_t)SQ.waves.size() * sizeof(hines::KCellWave));
  const int64_t sz_sb = al((int64_t)SQ.base.size() * sizeof(int64_t));
  const int64_t sz_sp = al((int64_t)SQ.pos.size() * sizeof(uint16_t));
  const int64_t sz_sc = al((int64_t)SQ.code.size() * sizeof(uint16_t));
  const int64_t sz_sm = al((int64_t)SQ.mbsrc.size() * sizeof(uint64_t));
  const hines::ResPlan& RP = P.res;
  const int64_t sz_rg = al((int64_t)RP.groups.size() * sizeof(hines::KResGroup));
  const int64_t sz_rl = al((int64_t)p->res_list.size() * sizeof(int32_t));
  const int64_t sz_rb = al((int64_t)RP.blob.size());
  const int64_t total = sz_br + sz_grp + sz_seg + sz_cell + sz_gl + sz_ws + sz_fl + sz_fm + sz_fp + sz_fa + sz_cw +
                        sz_cb + sz_cp + sz_cf + sz_cm + sz_cr + sz_cz + sz_sw + sz_sb + sz_sp + sz_sc + sz_sm +
                        sz_rg + sz_rl + sz_rb + 256;
  const int64_t scr_bytes = CL.nchunks * hines::kCellChunk * 64 * 16 + SQ.nchunks * hines::kSeqChunk * 64 * 16;
  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) e = static_scratch_init(p->device);
  if (e == hipSuccess) e = allow_lds(o.group_width);
  if (e == hipSuccess) e = res_class_attr();
  if (e == hipSuccess && P.res.built) {
    for (int k = 0; k < hines_plan::kResStreams && e == hipSuccess; ++k) {
      e = hipStreamCreateWithFlags(&p->res_streams[k], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&p->res_join[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->res_fork, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    delete p;
    return set_err(HINES_ERR_HIP, "device setup: %s", hipGetErrorString(e));
  }
  e = dev_alloc(&p->dev_mem, total);
  if (e != hipSuccess) {
    p->dev_mem = nullptr;
    delete p;
    return set_err(HINES_ERR_OOM, "device allocation of %lld bytes: %s", (long long)total, hipGetErrorString(e));
  }
  if (scr_bytes > 0) {
    e = dev_alloc(&p->scr_mem, scr_bytes);
    if (e != hipSuccess) {
      p->scr_mem = nullptr;
      dev_free(p->dev_mem, total);
      delete p;
      return set_err(HINES_ERR_OOM, "device allocation of %lld bytes for the cell-lane scratch: %s", (long long)scr_bytes,
                     hipGetErrorString(e));
    }
  }
  p->dev_bytes = total + scr_bytes;
  p->scr_bytes = scr_bytes;
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
  p->t.ws = P.ws_doubles > 0 ? (double*)(base + off) : nullptr;
  off += sz_ws;
  p->t.flow = (const hines::KFlow*)(base + off);
  if (e == hipSuccess) e = up(P.kflow.data(), (int64_t)P.kflow.size() * sizeof(hines::KFlow), off);
  off += sz_fl;
  p->t.fmask = (const uint64_t*)(base + off);
  if (e == hipSuccess) e = up(P.fmask.data(), (int64_t)P.fmask.size() * sizeof(uint64_t), off);
  off += sz_fm;
  p->t.fpos = (const uint16_t*)(base + off);
  if (e == hipSuccess) e = up(P.fpos.data(), (int64_t)P.fpos.size() * sizeof(uint16_t), off);
  off += sz_fp;
  p->t.faux = (const int16_t*)(base + off);
  if (e == hipSuccess) e = up(P.faux.data(), (int64_t)P.faux.size() * sizeof(int16_t), off);
  off += sz_fa;
  p->t.cwave = (const hines::KCellWave*)(base + off);
  if (e == hipSuccess) e = up(CL.waves.data(), (int64_t)CL.waves.size() * sizeof(hines::KCellWave), off);
  off += sz_cw;
  p->t.cbase = (const int64_t*)(base + off);
  if (e == hipSuccess) e = up(CL.base.data(), (int64_t)CL.base.size() * sizeof(int64_t), off);
  off += sz_cb;
  p->t.cpos = (const uint16_t*)(base + off);
  if (e == hipSuccess) e = up(CL.pos.data(), (int64_t)CL.pos.size() * sizeof(uint16_t), off);
  off += sz_cp;
  p->t.cflag = (const uint8_t*)(base + off);
  if (e == hipSuccess) e = up(CL.flags.data(), (int64_t)CL.flags.size(), off);
  off += sz_cf;
  p->t.cmsrc = (const uint64_t*)(base + off);
  if (e == hipSuccess) e = up(CL.mbsrc.data(), (int64_t)CL.mbsrc.size() * sizeof(uint64_t), off);
  off += sz_cm;
  p->t.crange = (const uint64_t*)(base + off);
  if (e == hipSuccess) e = up(CL.range.data(), (int64_t)CL.range.size() * sizeof(uint64_t), off);
  off += sz_cr;
  p->t.czero = sz_cz ? (double*)(base + off) : nullptr;
  if (e == hipSuccess && sz_cz) {
    static const double zeros[128] = {};
    e = up(zeros, sizeof(zeros), off);
  }
  off += sz_cz;
  p->t.swave = (const hines::KCellWave*)(base + off);
  if (e == hipSuccess) e = up(SQ.waves.data(), (int64_t)SQ.waves.size() * sizeof(hines::KCellWave), off);
  off += sz_sw;
  p->t.sbase = (const int64_t*)(base + off);
  if (e == hipSuccess) e = up(SQ.base.data(), (int64_t)SQ.base.size() * sizeof(int64_t), off);
  off += sz_sb;
  p->t.spos = (const uint16_t*)(base + off);
  if (e == hipSuccess) e = up(SQ.pos.data(), (int64_t)SQ.pos.size() * sizeof(uint16_t), off);
  off += sz_sp;
  p->t.scode = (const uint16_t*)(base + off);
  if (e == hipSuccess) e = up(SQ.code.data(), (int64_t)SQ.code.size() * sizeof(uint16_t), off);
  off += sz_sc;
  p->t.smsrc = (const uint64_t*)(base + off);
  if (e == hipSuccess) e = up(SQ.mbsrc.data(), (int64_t)SQ.mbsrc.size() * sizeof(uint64_t), off);
  off += sz_sm;
  p->t.rgrp = (const hines::KResGroup*)(base + off);
  if (e == hipSuccess) e = up(RP.groups.data(), (int64_t)RP.groups.size() * sizeof(hines::KResGroup), off);
  off += sz_rg;
  p->t.rlist = (const int32_t*)(base + off);
  if (e == hipSuccess) e = up(p->res_list.data(), (int64_t)p->res_list.size() * sizeof(int32_t), off);
  off += sz_rl;
  p->t.rblob = (const uint8_t*)(base + off);
  if (e == hipSuccess) e = up(RP.blob.data(), (int64_t)RP.blob.size(), off);
  off += sz_rb;
  p->t.cscr = (double*)p->scr_mem;
  p->t.cslots = CL.nchunks * hines::kCellChunk * 64;
  if (e != hipSuccess) {
    if (p->scr_mem) dev_free(p->scr_mem, scr_bytes);
    dev_free(p->dev_mem, total);
    delete p;
    return set_err(HINES_ERR_HIP, "table upload: %s", hipGetErrorString(e));
  }
  // the kernel tables now live on the device
  std::vector<KBranch>().swap(p->host.kbranch);
  if (!o.keep_tables) {
    std::vector<uint64_t>().swap(p->host.fmask);
    std::vector<uint16_t>().swap(p->host.fpos);
    std::vector<int16_t>().swap(p->host.faux);
    std::vector<uint16_t>().swap(p->host.cl.pos);
    std::vector<uint8_t>().swap(p->host.cl.flags);
    std::vector<uint16_t>().swap(p->host.sq.pos);
    std::vector<uint16_t>().swap(p->host.sq.code);
  }
  *out = p;
  return ok();
}

hines_status hines_solve(const hines_plan* p, const double* diag, const double* upper, const double* rhs, double* x,
                         int32_t ncells, void* stream) {
  hines_status st = check_call(p, ncells);
  if (st != HINES_OK) return st;
  if (p->host.n == 0) return ok();
  if (!diag || !upper || !rhs || !x) return set_err(HINES_ERR_NULL, "a device array is NULL");
  if ((const void*)x == (const void*)diag || (const void*)x == (const void*)upper)
    return set_err(HINES_ERR_STATE, "x must not alias diag or upper");
  RhsSpec rs{};
  rs.rhs = rhs;
  rs.mode = hdev::kRhsGiven;
  return run_solve(p, rs, diag, upper, x, stream);
}

hines_status hines_solve_noalloc(const hines_plan* p, const double* diag, const double* upper, const double* rhs,
                                 double* x, int32_t ncells, void* stream) {
  hines_status st = check_call(p, ncells);
  if (st != HINES_OK) return st;
  const bool seq = p->host.sq.built;  // index-order lanes, else depth-first ones
  if (!p->host.cl.built && !seq)
    return set_err(HINES_ERR_STATE, "hines_solve_noalloc needs a cell-lane plan (cell_lanes 1 or 2)");
  if (p->host.n == 0) return ok();
  if (!diag || !upper || !rhs || !x) return set_err(HINES_ERR_NULL, "a device array is NULL");
  if ((const void*)x == (const void*)diag || (const void*)x == (const void*)upper)
    return set_err(HINES_ERR_STATE, "x must not alias diag or upper");
  const int64_t need = seq ? p->host.sq.nchunks * hines::kSeqChunk * 64 * 16 : p->t.cslots * 16;
  if (need > kStaticScratchBytes)
    return set_err(HINES_ERR_TOO_BIG, "the plan's factors need %lld bytes; the static scratch holds %lld",
                   (long long)need, (long long)kStaticScratchBytes);
  void* ptr = static_scratch(p->device);
  if (!ptr) return set_err(HINES_ERR_STATE, "the static scratch of device %d is not resolved", p->device);
  DevTables t = p->t;
  t.cscr = (double*)ptr;
  RhsSpec rs{};
  rs.rhs = rhs;
  rs.mode = hdev::kRhsGiven;
  if (seq)
    hipLaunchKernelGGL(hdev::k_solve_seq<hdev::kFlowGiven>, dim3((unsigned)p->host.sq.nwaves), dim3(64), 0,
                       (hipStream_t)stream, t, rs, diag, upper, x);
  else
    hipLaunchKernelGGL(hdev::k_solve_cells<hdev::kFlowGiven>, dim3((unsigned)p->host.cl.nwaves), dim3(64), 0,
                       (hipStream_t)stream, t, rs, diag, upper, x);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(HINES_ERR_HIP, "launch: %s", hipGetErrorString(e));
  return ok();
}

hines_status hines_solve_mixed(const hines_plan* p, const float* diag32, const float* upper32, const double* rhs,
                               double* x, int32_t sweeps, int32_t ncells, void* stream) {
  hines_status st = check_call(p, ncells);
  if (st != HINES_OK) return st;
  if (sweeps < 0 || sweeps > 8) return set_err(HINES_ERR_OPTION, "sweeps must be in [0, 8]");
  if (p->host.n == 0) return ok();
  if (!diag32 || !upper32 || !rhs || !x) return set_err(HINES_ERR_NULL, "a device array is NULL");
  if (!p->mixed_ok)
    return set_err(HINES_ERR_TOO_BIG, "a group does not fit the FP32+refinement LDS image or the branch records");
  if ((const void*)x == (const void*)diag32 || (const void*)x == (const void*)upper32)
    return set_err(HINES_ERR_STATE, "x must not alias diag or upper");
  hipError_t e = launch_mixed(p, diag32, upper32, rhs, x, sweeps, (hipStream_t)stream);
  if (e != hipSuccess) return set_err(HINES_ERR_HIP, "launch: %s", hipGetErrorString(e));
  return ok();
}

hines_status hines_solve_stored32(const hines_plan* p, const float* diag32, const float* upper32, const double* rhs,
                                 double* x, int32_t ncells, void* stream) {
  hines_status st = check_call(p, ncells);
  if (st != HINES_OK) return st;
  if (!p->host.cl.built) return set_err(HINES_ERR_STATE, "hines_solve_stored32 needs a cell-lane plan");
  if (p->host.n == 0) return ok();
  if (!diag32 || !upper32 || !rhs || !x) return set_err(HINES_ERR_NULL, "a device array is NULL");
  if ((const void*)x == (const void*)diag32 || (const void*)x == (const void*)upper32)
    return set_err(HINES_ERR_STATE, "x must not alias diag or upper");
  RhsSpec rs{};
  rs.rhs = rhs;
  rs.mode = hdev::kRhsGiven;
  hipLaunchKernelGGL((hdev::k_solve_cells<hdev::kFlowGiven, float>), dim3((unsigned)p->host.cl.nwaves), dim3(64), 0,
                     (hipStream_t)stream, p->t, rs, diag32, upper32, x);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(HINES_ERR_HIP, "launch: %s", hipGetErrorString(e));
  return ok();
}

hines_status hines_timestep_assembled(const hines_plan* p, const double* g, const double* upper, const double* c,
                                     const double* ge, const double* v_in, double* v_out, int32_t ncells,
                                     void* stream) {
  hines_status st = check_call(p, ncells);
  if (st != HINES_OK) return st;
  if (!p->host.cl.built) return set_err(HINES_ERR_STATE, "hines_timestep_assembled needs a cell-lane plan");
  if (p->host.n == 0) return ok();
  if (!g || !upper || !c || !ge || !v_in || !v_out) return set_err(HINES_ERR_NULL, "a device array is NULL");
  const void* o = v_out;
  if (o == g || o == upper || o == c || o == ge) return set_err(HINES_ERR_STATE, "v_out may alias only v_in");
  RhsSpec rs{};
  rs.c = c;
  rs.v = v_in;
  rs.icur = ge;
  rs.mode = hdev::kRhsCV;
  hipLaunchKernelGGL((hdev::k_solve_cells<hdev::kCellCond, double>), dim3((unsigned)p->host.cl.nwaves), dim3(64), 0,
                     (hipStream_t)stream, p->t, rs, g, upper, v_out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(HINES_ERR_HIP, "launch: %s", hipGetErrorString(e));
  return ok();
}

hines_status hines_timestep(const hines_plan* p, const double* diag, const double* upper, const double* c,
                            const double* v_in, double* v_out, const double* i_inj, double noise_sigma,
                            uint32_t noise_seed, uint32_t step, int32_t ncells, void* stream) {
  hines_status st = check_call(p, ncells);
  if (st != HINES_OK) return st;
  if (p->host.n == 0) return ok();
  if (!diag || !upper || !c || !v_in || !v_out) return set_err(HINES_ERR_NULL, "a device array is NULL");
  const void* o = v_out;
  if (o == diag || o == upper || o == c || (i_inj && o == i_inj))
    return set_err(HINES_ERR_STATE, "v_out may alias only v_in");
  RhsSpec rs{};
  rs.c = c;
  rs.v = v_in;
  rs.icur = i_inj;
  rs.sigma = noise_sigma;
  rs.seed = noise_seed;
  rs.step = step;
  rs.mode = (i_inj == nullptr && noise_sigma != 0.0) ? hdev::kRhsNoise : hdev::kRhsCV;
  return run_solve(p, rs, diag, upper, v_out, stream);
}

hines_status hines_timeloop_create(const hines_plan* p, const double* diag, const double* upper, const double* c,
                                   double* v, const double* i_inj, double noise_sigma, uint32_t noise_seed,
                                   uint32_t first_step, int32_t nsteps, int32_t ncells, hines_timeloop** out) {
  if (!out) return set_err(HINES_ERR_NULL, "out is NULL");
  *out = nullptr;
  hines_status st = check_call(p, ncells);
  if (st != HINES_OK) return st;
  if (nsteps < 1) return set_err(HINES_ERR_OPTION, "nsteps must be >= 1");
  if (p->host.n == 0) {  // nothing to step: a loop without a graph, launch does nothing
    *out = new (std::nothrow) hines_timeloop();
    if (!*out) return set_err(HINES_ERR_OOM, "host allocation failed");
    (*out)->nsteps = nsteps;
    return ok();
  }
  if (!diag || !upper || !c || !v) return set_err(HINES_ERR_NULL, "a device array is NULL");
  const void* vo = v;
  if (vo == diag || vo == upper || vo == c || (i_inj && vo == i_inj))
    return set_err(HINES_ERR_STATE, "v must not alias the matrix, c or the current");
  hines_timeloop* tl = new (std::nothrow) hines_timeloop();
  if (!tl) return set_err(HINES_ERR_OOM, "host allocation failed");
  const bool noise = i_inj == nullptr && noise_sigma != 0.0;
  // cell-lane plans keep the factors: per launch, factor A and move c, the
  // current and V into the walk layout; K steps there; V back at the end
  bool factored = p->host.cl.built && p->host.n > 0;
  hdev::CellLoop L{};
  if (factored) {
    const int64_t S = p->t.cslots;
    // f, 1 / d', c, the current, V; positions for the draws
    const int64_t bytes = 8 * S * (i_inj ? 5 : 4) + (noise ? 2 * S : 0) + 256;
    if (dev_alloc(&tl->mem, bytes) != hipSuccess) {
      (void)hipGetLastError();  // no room for the factors: capture the plain steps instead
      tl->mem = nullptr;
      factored = false;
    } else {
      tl->bytes = bytes;
    }
  }
  if (factored) {
    const int64_t S = p->t.cslots;
    double* m = (double*)tl->mem;
    L.f = m;
    L.r = m + S;
    L.c = m + 2 * S;
    L.v = m + 3 * S;
    L.ci = i_inj ? m + 4 * S : nullptr;
    L.lp = noise ? (const uint16_t*)(m + 4 * S) : nullptr;
    L.sigma = noise_sigma;
    L.seed = noise_seed;
  }
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  const bool capturing = e == hipSuccess;
  if (factored && e == hipSuccess) {
    const dim3 grid((unsigned)p->host.cl.nwaves);
    if (noise)
      hipLaunchKernelGGL(hdev::k_cells_lane_pos, grid_for(p->t.cslots, 256), dim3(256), 0, cs, p->t,
                         (uint16_t*)L.lp, p->host.cl.nchunks);
    RhsSpec rs0{};
    hipLaunchKernelGGL(hdev::k_solve_cells<hdev::kCellFactor>, grid, dim3(64), 0, cs, p->t, rs0, diag, upper,
                       (double*)L.f);  // f at L.f, 1 / d' at L.f + slots = L.r
    hipLaunchKernelGGL(hdev::k_cells_to_walk, grid, dim3(64), 0, cs, p->t, c, (double*)L.c);
    if (i_inj) hipLaunchKernelGGL(hdev::k_cells_to_walk, grid, dim3(64), 0, cs, p->t, i_inj, (double*)L.ci);
    hipLaunchKernelGGL(hdev::k_cells_to_walk, grid, dim3(64), 0, cs, p->t, (const double*)v, L.v);
    for (int32_t k = 0; k < nsteps; ++k) {
      L.step = first_step + (uint32_t)k;
      if (noise)
        hipLaunchKernelGGL(hdev::k_cells_step<hdev::kFlowNoise>, grid, dim3(64), 0, cs, p->t, L);
      else if (i_inj)
        hipLaunchKernelGGL(hdev::k_cells_step<hdev::kFlowCVI>, grid, dim3(64), 0, cs, p->t, L);
      else
        hipLaunchKernelGGL(hdev::k_cells_step<hdev::kFlowCV>, grid, dim3(64), 0, cs, p->t, L);
    }
    hipLaunchKernelGGL(hdev::k_cells_from_walk, grid, dim3(64), 0, cs, p->t, (const double*)L.v, v);
    e = hipGetLastError();
  }
  for (int32_t k = 0; k < nsteps && e == hipSuccess && p->host.n > 0 && !factored; ++k) {
    RhsSpec rs{};
    rs.c = c;
    rs.v = v;
    rs.icur = i_inj;
    rs.sigma = noise_sigma;
    rs.seed = noise_seed;
    rs.step = first_step + (uint32_t)k;
    rs.mode = (i_inj == nullptr && noise_sigma != 0.0) ? hdev::kRhsNoise : hdev::kRhsCV;
    e = launch_solve(p, rs, diag, upper, v, cs);
  }
  if (capturing) {
    hipError_t e2 = hipStreamEndCapture(cs, &tl->graph);
    if (e == hipSuccess) e = e2;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&tl->exec, tl->graph, nullptr, nullptr, 0);
  if (cs) hipStreamDestroy(cs);
  if (e != hipSuccess) {
    if (tl->exec) hipGraphExecDestroy(tl->exec);
    if (tl->graph) hipGraphDestroy(tl->graph);
    if (tl->mem) dev_free(tl->mem, tl->bytes);
    delete tl;
    return set_err(HINES_ERR_HIP, "time loop capture: %s", hipGetErrorString(e));
  }
  tl->nsteps = nsteps;
  *out = tl;
  return ok();
}

hines_status hines_timeloop_launch(hines_timeloop* tl, void* stream) {
  if (!tl) return set_err(HINES_ERR_NULL, "time loop is NULL");
  if (!tl->exec) return ok();  // empty plan
  hipError_t e = hipGraphLaunch(tl->exec, (hipStream_t)stream);
  if (e != hipSuccess) return set_err(HINES_ERR_HIP, "graph launch: %s", hipGetErrorString(e));
  return ok();
}

hines_status hines_timeloop_destroy(hines_timeloop* tl) {
  if (!tl) return ok();
  hipError_t e = hipSuccess;
  if (tl->exec) e = hipGraphExecDestroy(tl->exec);
  if (tl->graph) {
    hipError_t e2 = hipGraphDestroy(tl->graph);
    if (e == hipSuccess) e = e2;
  }
  if (tl->mem) {
    hipError_t e2 = dev_free(tl->mem, tl->bytes);  // waits for the device
    if (e == hipSuccess) e = e2;
  }
  delete tl;
  if (e != hipSuccess) return set_err(HINES_ERR_HIP, "time loop destroy: %s", hipGetErrorString(e));
  return ok();
}

hines_status hines_assemble(hines_plan* p, const double* a, const double* c, double* diag, double* upper,
                            void* stream) {
  hines_status st = check_call(p, p ? (int32_t)p->host.ncells : 0);
  if (st != HINES_OK) return st;
  if (p->host.n == 0) return ok();
  if (!a || !c || !diag || !upper) return set_err(HINES_ERR_NULL, "a device array is NULL");
  st = ensure_adjoint_tables(p);
  if (st != HINES_OK) return st;
  const int64_t n = p->host.n;
  hipLaunchKernelGGL(hdev::k_assemble, grid_for(n, 256), dim3(256), 0, (hipStream_t)stream, n, p->d_parent,
                     p->d_ch_off, p->d_ch, a, c, diag, upper);
  return launched();
}

hines_status hines_gather_roots(hines_plan* p, const double* v, double* out, void* stream) {
  hines_status st = check_call(p, p ? (int32_t)p->host.ncells : 0);
  if (st != HINES_OK) return st;
  if (p->host.ncells == 0) return ok();
  if (!v || !out) return set_err(HINES_ERR_NULL, "a device array is NULL");
  st = ensure_adjoint_tables(p);
  if (st != HINES_OK) return st;
  const int32_t nc = (int32_t)p->host.ncells;
  hipLaunchKernelGGL(hdev::k_gather_roots, grid_for(nc, 256), dim3(256), 0, (hipStream_t)stream, nc, p->d_cell_off,
                     v, out);
  return launched();
}

hines_status hines_adjoint_rhs(hines_plan* p, const double* c, const double* lam_next, const double* g_roots,
                               double* mu, void* stream) {
  hines_status st = check_call(p, p ? (int32_t)p->host.ncells : 0);
  if (st != HINES_OK) return st;
  if (p->host.n == 0) return ok();
  if (!c || !g_roots || !mu) return set_err(HINES_ERR_NULL, "a device array is NULL");
  st = ensure_adjoint_tables(p);
  if (st != HINES_OK) return st;
  const int64_t n = p->host.n;
  hipLaunchKernelGGL(hdev::k_adjoint_rhs, grid_for(n, 256), dim3(256), 0, (hipStream_t)stream, n, p->d_parent,
                     p->d_cell_off, (int32_t)p->host.ncells, c, lam_next, g_roots, mu);
  return launched();
}

hines_status hines_adjoint_accumulate(hines_plan* p, const double* lam, const double* v, const double* v_prev,
                                      double* grad_a, double* grad_c, double* grad_i, void* stream) {
  hines_status st = check_call(p, p ? (int32_t)p->host.ncells : 0);
  if (st != HINES_OK) return st;
  if (p->host.n == 0) return ok();
  if (!lam || !v || !v_prev || !grad_a || !grad_c || !grad_i)
    return set_err(HINES_ERR_NULL, "a device array is NULL");
  st = ensure_adjoint_tables(p);
  if (st != HINES_OK) return st;
  const int64_t n = p->host.n;
  hipLaunchKernelGGL(hdev::k_adjoint_accumulate, grid_for(n, 256), dim3(256), 0, (hipStream_t)stream, n,
                     p->d_parent, lam, v, v_prev, grad_a, grad_c, grad_i);
  return launched();
}

hines_status hines_layout_size(const hines_plan* p, int64_t* slots) {
  if (!p || !slots) return set_err(HINES_ERR_NULL, "NULL argument");
  *slots = 0;
  if (!p->host.cl.built) return set_err(HINES_ERR_STATE, "the solver layout needs a cell-lane plan");
  *slots = p->host.cl.nchunks * hines::kCellChunk * 64;
  return ok();
}

static hines_status layout_call(const hines_plan* p, const void* a, const void* b) {
  hines_status st = check_call(p, p ? (int32_t)p->host.ncells : 0);
  if (st != HINES_OK) return st;
  if (!p->host.cl.built) return set_err(HINES_ERR_STATE, "the solver layout needs a cell-lane plan");
  if (p->host.n > 0 && (!a || !b)) return set_err(HINES_ERR_NULL, "a device array is NULL");
  if (p->host.n > 0 && a == b) return set_err(HINES_ERR_STATE, "src and dst must not alias");
  return HINES_OK;
}

hines_status hines_to_layout(const hines_plan* p, const double* src, double* dst, void* stream) {
  hines_status st = layout_call(p, src, dst);
  if (st != HINES_OK) return st;
  if (p->host.n == 0) return ok();
  hipLaunchKernelGGL(hdev::k_cells_to_walk, dim3((unsigned)p->host.cl.nwaves), dim3(64), 0, (hipStream_t)stream,
                     p->t, src, dst);
  return launched();
}

hines_status hines_from_layout(const hines_plan* p, const double* src, double* dst, void* stream) {
  hines_status st = layout_call(p, src, dst);
  if (st != HINES_OK) return st;
  if (p->host.n == 0) return ok();
  hipLaunchKernelGGL(hdev::k_cells_from_walk, dim3((unsigned)p->host.cl.nwaves), dim3(64), 0, (hipStream_t)stream,
                     p->t, src, dst);
  return launched();
}

hines_status hines_solve_layout(const hines_plan* p, const double* diag_l, const double* upper_l,
                                const double* rhs_l, double* x_l, int32_t ncells, void* stream) {
  hines_status st = check_call(p, ncells);
  if (st != HINES_OK) return st;
  if (!p->host.cl.built) return set_err(HINES_ERR_STATE, "hines_solve_layout needs a cell-lane plan");
  if (p->host.n == 0) return ok();
  if (!diag_l || !upper_l || !rhs_l || !x_l) return set_err(HINES_ERR_NULL, "a device array is NULL");
  if ((const void*)x_l == (const void*)diag_l || (const void*)x_l == (const void*)upper_l)
    return set_err(HINES_ERR_STATE, "x must not alias diag or upper");
  hdev::WalkSolve L{diag_l, upper_l, rhs_l, x_l, p->t.cscr};
  hipLaunchKernelGGL(hdev::k_solve_walk, dim3((unsigned)p->host.cl.nwaves), dim3(64), 0, (hipStream_t)stream, p->t,
                     L);
  return launched();
}

hines_status hines_check_matrix(hines_plan* p, const double* diag, const double* upper, int64_t* first_bad,
                                void* stream) {
  if (first_bad) *first_bad = -1;
  hines_status st = check_call(p, p ? (int32_t)p->host.ncells : 0);
  if (st != HINES_OK) return st;
  if (p->host.n == 0) return ok();
  if (!diag || !upper) return set_err(HINES_ERR_NULL, "a device array is NULL");
  st = ensure_adjoint_tables(p);
  if (st != HINES_OK) return st;
  const int64_t n = p->host.n;
  const hipStream_t s = (hipStream_t)stream;
  const unsigned long long none = ~0ull;
  hipLaunchKernelGGL(hdev::k_fill_u64, dim3(1), dim3(64), 0, s, p->d_flag, none);
  hipLaunchKernelGGL(hdev::k_check_sdd, grid_for(n, 256), dim3(256), 0, s, n, p->d_parent, p->d_ch_off, p->d_ch,
                     diag, upper, p->d_flag);
  unsigned long long bad = none;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, p->d_flag, sizeof bad, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_err(HINES_ERR_HIP, "matrix check: %s", hipGetErrorString(e));
  if (bad == none) return ok();
  if (first_bad) *first_bad = (int64_t)bad;
  return set_err(HINES_ERR_NOT_SDD, "row %lld is not strictly diagonally dominant with a positive diagonal",
                 (long long)bad);
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
  info->kernel = p->host.sq.built ? 5
                 : p->host.res.built ? 4
                 : p->host.cl.built ? 3
                                    : (p->host.flow ? 1 : (p->host.opt.bitwise ? 2 : 0));
  if (p->host.cl.built || p->host.sq.built) info->nclasses = 1;
  if (p->host.res.built) info->nclasses = (int32_t)p->res_buckets.size();
  int32_t mk = 0;
  int64_t ng_ws = 0;
  for (const auto& G : p->host.kgroup) {
    if (p->host.flow && G.ws_off < 0) mk = std::max(mk, G.makespan);
    ng_ws += G.ws_off >= 0;
  }
  if (p->host.cl.built)
    for (const auto& W : p->host.cl.waves) mk = std::max(mk, W.nchunk);
  if (p->host.sq.built)
    for (const auto& W : p->host.sq.waves) mk = std::max(mk, W.nchunk);
  if (p->host.res.built) {
    mk = 0;
    for (const auto& G : p->host.res.groups) mk = std::max(mk, G.nchunk * hines::kResK);
  }
  info->max_makespan = mk;
  info->workspace_groups = ng_ws;
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
  if (p->dev_mem || p->adj_mem || p->scr_mem) {
    int prev = -1;
    hipGetDevice(&prev);
    if (prev != p->device) hipSetDevice(p->device);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess && p->dev_mem) e = dev_free(p->dev_mem, p->dev_bytes - p->scr_bytes);
    if (e == hipSuccess && p->scr_mem) e = dev_free(p->scr_mem, p->scr_bytes);
    if (e == hipSuccess && p->adj_mem) e = dev_free(p->adj_mem, p->adj_bytes);
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
    case HINES_ERR_NCELLS: return "cell count mismatch";
    case HINES_ERR_OPTION: return "bad option";
    case HINES_ERR_OOM: return "out of memory";
    case HINES_ERR_HIP: return "HIP error";
    case HINES_ERR_TOO_BIG: return "group too big";
    case HINES_ERR_NOT_SDD: return "matrix not strictly diagonally dominant";
    case HINES_ERR_STATE: return "invalid state";
  }
  return "unknown status";
}

const char* hines_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
