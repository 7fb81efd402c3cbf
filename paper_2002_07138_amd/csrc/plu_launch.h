// Launch machinery shared by every kernel of libpowerlu.
//
// Each kernel is written as a body  void body(const Args&, const Grid&)  that
// sees its block index and grid through Grid instead of blockIdx/gridDim.
// The same body then runs
//   * alone:   k_one<...>  with the hardware grid (one problem), or
//   * grouped: k_group<...> where the problems of a batch own consecutive
//              ranges of virtual blocks of one launch; a persistent 1-D grid
//              walks the virtual blocks, each finding its problem by binary
//              search over the range starts.
// dispatch() launches a body alone, or, while a Recorder is installed on the
// calling thread, records the launch (arguments by value, its grid, and the
// grouped launcher of the same body) so that a batch executor can merge the
// launches of many problems into grouped launches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <vector>

namespace plu {

struct Grid {
  uint32_t bx, by, gx, gy;
};

__device__ __forceinline__ Grid hw_grid() {
  return Grid{blockIdx.x, blockIdx.y, gridDim.x, gridDim.y};
}

struct GroupDim {
  uint32_t gx, gy;
};

template <class Args, void (*Body)(const Args&, const Grid&), int NTHR, int MINW>
__global__ __launch_bounds__(NTHR, MINW) void k_one(Args a) {
  Body(a, hw_grid());
}

template <class Args, void (*Body)(const Args&, const Grid&), int NTHR, int MINW>
__global__ __launch_bounds__(NTHR, MINW) void k_group(const Args* __restrict__ tab,
                                                      const GroupDim* __restrict__ dims,
                                                      const uint32_t* __restrict__ start, int n) {
  const uint32_t total = start[n];
  for (uint32_t v = blockIdx.x; v < total; v += gridDim.x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (start[mid] <= v) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t local = v - start[lo];
    const GroupDim d = dims[lo];
    const Grid g{local % d.gx, local / d.gx, d.gx, d.gy};
    const Args a = tab[lo];
    Body(a, g);
    __syncthreads();   // the next virtual block reuses the LDS of this one
  }
}

// Grouped cooperative launch: exactly one virtual block per workgroup (all
// resident at once), no persistent loop.
template <class Args, void (*Body)(const Args&, const Grid&), int NTHR, int MINW>
__global__ __launch_bounds__(NTHR, MINW) void k_group_coop(const Args* __restrict__ tab,
                                                           const GroupDim* __restrict__ dims,
                                                           const uint32_t* __restrict__ start,
                                                           int n) {
  const uint32_t v = blockIdx.x;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= v) lo = mid;
    else hi = mid - 1;
  }
  const uint32_t local = v - start[lo];
  const GroupDim d = dims[lo];
  const Args a = tab[lo];   // by value: uniform, kept in scalar registers
  Body(a, Grid{local % d.gx, local / d.gx, d.gx, d.gy});
}

// One recorded launch of a body.
struct LaunchRec {
  const void* key;                 // identifies the body (its grouped kernel)
  std::vector<unsigned char> args;
  uint32_t gx, gy;
  size_t dynlds;
  bool coop;
  int nthr;
  // launches the grouped kernel of this body over a device table of n
  // argument blocks (sizeof args each), their grids and range starts
  hipError_t (*grouped)(const void* tab, const GroupDim* dims, const uint32_t* start, int n,
                        uint32_t total, size_t dynlds, bool coop, hipStream_t s);
};

struct Recorder {
  std::vector<LaunchRec> ops;
};

// The recorder of the calling thread (nullptr: launches run immediately).
Recorder*& thread_recorder();

hipError_t set_dynamic_lds(const void* fn, size_t bytes);

// Whether the kernels whose workgroups wait on each other (the LU panel) go
// out as cooperative launches (PLU_COOP_LAUNCH=1) or as ordinary ones (the
// default).  A cooperative launch waits for the device to drain the other
// queues' work, which cost about 30 us per panel and kept panels from
// overlapping other streams' kernels.  An ordinary launch relies on the
// grid's workgroups all becoming resident: they are few (at most 64 of 512
// threads per panel, and the batched path keeps the panels in flight within
// one per CU), every other kernel's workgroups finish on their own and free
// their slots, and every wait in the panel is bounded in time (a starved
// panel returns PLU_ERR_TIMEOUT, it does not hang).
bool coop_launch();

// Pinned host staging and device copy of the argument tables of a merged
// launch sequence (owned by a handle; grown on demand).
struct MergeBuffers {
  unsigned char* host = nullptr;
  unsigned char* dev = nullptr;
  size_t cap = 0;
  hipEvent_t copied = nullptr;   // recorded after each table copy
  bool copied_pending = false;
  bool capturing = false;        // inside a graph capture: no event records
  hipError_t reserve(size_t bytes);
  void release();
  void destroy();
};

struct MergeStats {
  size_t recorded = 0;   // launches the problems would have made one by one
  size_t launches = 0;   // grouped launches actually made
};

// Runs the recorded launch lists of several independent problems on stream
// s: each list in order, with launches of the same kernel body from
// different lists merged into grouped launches (cooperative ones split so
// that at most coop_cap workgroups are resident at once).
hipError_t run_merged(const std::vector<const Recorder*>& lists, hipStream_t s, int coop_cap,
                      MergeBuffers& buf, MergeStats* stats);
// Incremental form: advances head[i] (the next op of list i) through at
// most max_groups grouped launches.
hipError_t run_merged_steps(const std::vector<const Recorder*>& lists, std::vector<size_t>& head,
                            hipStream_t s, int coop_cap, size_t max_groups, MergeBuffers& buf,
                            MergeStats* stats);
// Bytes of argument tables run_merged needs for these lists.
size_t merged_table_bytes(const std::vector<const Recorder*>& lists, int coop_cap);

template <class Args, void (*Body)(const Args&, const Grid&), int NTHR, int MINW>
hipError_t launch_grouped(const void* tab, const GroupDim* dims, const uint32_t* start, int n,
                          uint32_t total, size_t dynlds, bool coop, hipStream_t s) {
  const Args* t = reinterpret_cast<const Args*>(tab);
  if (coop) {
    // every virtual block of a cooperative body must be resident at once
    const void* fc = reinterpret_cast<const void*>(&k_group_coop<Args, Body, NTHR, MINW>);
    if (dynlds > 65536) {
      hipError_t e = set_dynamic_lds(fc, dynlds);
      if (e != hipSuccess) return e;
    }
    if (!coop_launch()) {
      hipLaunchKernelGGL((k_group_coop<Args, Body, NTHR, MINW>), dim3(total), dim3(NTHR), dynlds,
                         s, t, dims, start, n);
      return hipGetLastError();
    }
    void* params[] = {(void*)&t, (void*)&dims, (void*)&start, (void*)&n};
    return hipLaunchCooperativeKernel(fc, dim3(total), dim3(NTHR), params, (unsigned)dynlds, s);
  }
  const void* fn = reinterpret_cast<const void*>(&k_group<Args, Body, NTHR, MINW>);
  if (dynlds > 65536) {
    hipError_t e = set_dynamic_lds(fn, dynlds);
    if (e != hipSuccess) return e;
  }
  const uint32_t grid = total < 8192u ? total : 8192u;
  hipLaunchKernelGGL((k_group<Args, Body, NTHR, MINW>), dim3(grid), dim3(NTHR), dynlds, s, t,
                     dims, start, n);
  return hipGetLastError();
}

template <class Args, void (*Body)(const Args&, const Grid&), int NTHR, int MINW = 1>
hipError_t dispatch(const Args& a, dim3 grid, size_t dynlds, hipStream_t s, bool coop = false) {
  if (grid.x == 0 || grid.y == 0) return hipSuccess;
  if (Recorder* r = thread_recorder()) {
    LaunchRec rec;
    rec.key = reinterpret_cast<const void*>(&k_group<Args, Body, NTHR, MINW>);
    rec.args.resize(sizeof(Args));
    std::memcpy(rec.args.data(), &a, sizeof(Args));
    rec.gx = grid.x;
    rec.gy = grid.y;
    rec.dynlds = dynlds;
    rec.coop = coop;
    rec.nthr = NTHR;
    rec.grouped = &launch_grouped<Args, Body, NTHR, MINW>;
    r->ops.push_back(std::move(rec));
    return hipSuccess;
  }
  const void* fn = reinterpret_cast<const void*>(&k_one<Args, Body, NTHR, MINW>);
  if (dynlds > 65536) {
    hipError_t e = set_dynamic_lds(fn, dynlds);
    if (e != hipSuccess) return e;
  }
  if (coop && coop_launch()) {
    void* params[] = {(void*)&a};
    return hipLaunchCooperativeKernel(fn, grid, dim3(NTHR), params, (unsigned)dynlds, s);
  }
  hipLaunchKernelGGL((k_one<Args, Body, NTHR, MINW>), grid, dim3(NTHR), dynlds, s, a);
  return hipGetLastError();
}

}  // namespace plu
