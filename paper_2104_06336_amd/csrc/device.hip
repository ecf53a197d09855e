// Per-device runtime queries shared by the launchers.
#include <mutex>
#include <vector>

#include "common.h"

namespace stem {

namespace {
struct ResidentEntry {
  const void* fn;
  int dev, threads;
  size_t lds;
  int blocks;
};
std::mutex g_resident_mu;
std::vector<ResidentEntry> g_resident;
}  // namespace

int resident_blocks(const void* fn, int threads, size_t lds) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  {
    std::lock_guard<std::mutex> lk(g_resident_mu);
    for (const ResidentEntry& e : g_resident)
      if (e.fn == fn && e.dev == dev && e.threads == threads && e.lds == lds) return e.blocks;
  }
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, threads, lds) != hipSuccess) return 0;
  const int blocks = cus * per;
  std::lock_guard<std::mutex> lk(g_resident_mu);
  g_resident.push_back(ResidentEntry{fn, dev, threads, lds, blocks});
  return blocks;
}

}  // namespace stem
