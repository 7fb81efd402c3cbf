// Batched execution: many PowerLU / PowerLU_FP problems of uneven shapes in
// grouped launches (the same kernel bodies as the single-problem path, with
// the problems of a batch owning consecutive ranges of virtual blocks).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <mutex>
#include <unordered_set>

#include "plu_internal.h"

namespace plu {

Recorder*& thread_recorder() {
  static thread_local Recorder* r = nullptr;
  return r;
}

bool coop_launch() {
  static const bool on = [] {
    const char* e = std::getenv("PLU_COOP_LAUNCH");
    return e && e[0] == '1';
  }();
  return on;
}

hipError_t set_dynamic_lds(const void* fn, size_t bytes) {
  // the attribute is per kernel; set it once per (kernel, size)
  static std::mutex mu;
  static std::unordered_set<const void*> done;
  std::lock_guard<std::mutex> lk(mu);
  if (done.count(fn)) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) done.insert(fn);
  return e;
}

}  // namespace plu

namespace plu {

namespace {

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Group {
  const LaunchRec* first;
  std::vector<const LaunchRec*> recs;
  size_t args_off = 0, dims_off = 0, start_off = 0;
  uint32_t total = 0;
  size_t dynlds = 0;
};

// The merge plan: repeatedly launch the kernel body that heads the most
// lists; cooperative groups are split at the residency limit.  Fills the
// table offsets and returns the table size in bytes.
size_t plan_groups(const std::vector<const Recorder*>& lists, std::vector<size_t>& head,
                   int coop_cap, size_t max_groups, std::vector<Group>& groups) {
  while (groups.size() < max_groups) {
    std::vector<std::pair<const void*, int>> counts;
    for (size_t i = 0; i < lists.size(); ++i) {
      if (head[i] >= lists[i]->ops.size()) continue;
      const void* k = lists[i]->ops[head[i]].key;
      bool found = false;
      for (auto& c : counts)
        if (c.first == k) {
          ++c.second;
          found = true;
          break;
        }
      if (!found) counts.push_back({k, 1});
    }
    if (counts.empty()) break;
    auto best = counts[0];
    for (auto& c : counts)
      if (c.second > best.second) best = c;
    Group g;
    g.first = nullptr;
    for (size_t i = 0; i < lists.size(); ++i) {
      if (head[i] >= lists[i]->ops.size()) continue;
      const LaunchRec& r = lists[i]->ops[head[i]];
      if (r.key != best.first) continue;
      const uint32_t nb = r.gx * r.gy;
      if (r.coop && g.first && g.total + nb > (uint32_t)coop_cap) {
        groups.push_back(std::move(g));
        g = Group();
        g.first = nullptr;
      }
      if (!g.first) g.first = &r;
      g.recs.push_back(&r);
      g.total += nb;
      if (r.dynlds > g.dynlds) g.dynlds = r.dynlds;
      ++head[i];
    }
    groups.push_back(std::move(g));
  }
  size_t off = 0;
  for (auto& g : groups) {
    const size_t asz = g.first->args.size();
    g.args_off = off;
    off = align256(off + asz * g.recs.size());
    g.dims_off = off;
    off = align256(off + sizeof(GroupDim) * g.recs.size());
    g.start_off = off;
    off = align256(off + sizeof(uint32_t) * (g.recs.size() + 1));
  }
  return off;
}

}  // namespace

size_t merged_table_bytes(const std::vector<const Recorder*>& lists, int coop_cap) {
  std::vector<Group> groups;
  std::vector<size_t> head(lists.size(), 0);
  return plan_groups(lists, head, coop_cap, SIZE_MAX, groups);
}

hipError_t run_merged(const std::vector<const Recorder*>& lists, hipStream_t s, int coop_cap,
                      MergeBuffers& buf, MergeStats* stats) {
  std::vector<size_t> head(lists.size(), 0);
  return run_merged_steps(lists, head, s, coop_cap, SIZE_MAX, buf, stats);
}

hipError_t run_merged_steps(const std::vector<const Recorder*>& lists, std::vector<size_t>& head,
                            hipStream_t s, int coop_cap, size_t max_groups, MergeBuffers& buf,
                            MergeStats* stats) {
  std::vector<Group> groups;
  const size_t off = plan_groups(lists, head, coop_cap, max_groups, groups);
  if (groups.empty()) return hipSuccess;
  // argument tables in one host staging buffer, copied to the device once
  hipError_t e;
  if ((e = buf.reserve(off)) != hipSuccess) return e;
  // the previous sequence's table copy must have left the staging buffer
  if (buf.copied_pending) {
    if ((e = hipEventSynchronize(buf.copied)) != hipSuccess) return e;
    buf.copied_pending = false;
  }
  unsigned char* hb = buf.host;
  for (auto& g : groups) {
    const size_t asz = g.first->args.size();
    GroupDim* dims = reinterpret_cast<GroupDim*>(hb + g.dims_off);
    uint32_t* start = reinterpret_cast<uint32_t*>(hb + g.start_off);
    uint32_t acc = 0;
    for (size_t j = 0; j < g.recs.size(); ++j) {
      const LaunchRec* r = g.recs[j];
      if (r->args.size() != asz) return hipErrorInvalidValue;
      std::memcpy(hb + g.args_off + j * asz, r->args.data(), asz);
      dims[j] = GroupDim{r->gx, r->gy};
      start[j] = acc;
      acc += r->gx * r->gy;
    }
    start[g.recs.size()] = acc;
  }
  if (off > 0) {
    if ((e = hipMemcpyAsync(buf.dev, buf.host, off, hipMemcpyHostToDevice, s)) != hipSuccess)
      return e;
    if (!buf.capturing) {
      if ((e = hipEventRecord(buf.copied, s)) != hipSuccess) return e;
      buf.copied_pending = true;
    }
  }
  // grouped launches
  for (auto& g : groups) {
    const unsigned char* db = buf.dev;
    if ((e = g.first->grouped(db + g.args_off, reinterpret_cast<const GroupDim*>(db + g.dims_off),
                              reinterpret_cast<const uint32_t*>(db + g.start_off),
                              (int)g.recs.size(), g.total, g.dynlds, g.first->coop, s)) !=
        hipSuccess)
      return e;
  }
  if (stats) {
    stats->launches += groups.size();
    for (auto& g : groups) stats->recorded += g.recs.size();
  }
  return hipSuccess;
}

hipError_t MergeBuffers::reserve(size_t bytes) {
  if (!copied) {
    hipError_t e = hipEventCreateWithFlags(&copied, hipEventDisableTiming);
    if (e != hipSuccess) {
      copied = nullptr;
      return e;
    }
  }
  if (bytes <= cap) return hipSuccess;
  // the previous tables may still be read by queued copies: wait for them
  if (host || dev) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
  }
  release();
  size_t c = bytes + bytes / 2 + 4096;
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&host), c, hipHostMallocDefault);
  if (e != hipSuccess) {
    host = nullptr;
    return e;
  }
  e = hipMalloc(reinterpret_cast<void**>(&dev), c);
  if (e != hipSuccess) {
    (void)hipHostFree(host);
    host = nullptr;
    dev = nullptr;
    return e;
  }
  cap = c;
  return hipSuccess;
}

void MergeBuffers::release() {
  if (host) (void)hipHostFree(host);
  if (dev) (void)hipFree(dev);
  host = nullptr;
  dev = nullptr;
  cap = 0;
}

void MergeBuffers::destroy() {
  if (copied_pending) (void)hipEventSynchronize(copied);
  release();
  if (copied) (void)hipEventDestroy(copied);
  copied = nullptr;
  copied_pending = false;
}

}  // namespace plu
