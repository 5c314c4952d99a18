// Host-to-device uploads of small host tables (series plans, sketch
// coefficients) that a HIP graph may capture.
//
// A captured memcpy node reads its host source again at every replay, so the
// source must outlive the graph and never change.  Every uploaded table is
// therefore also kept, once per distinct content, in pinned host memory owned
// by the library for the life of the process (up to kPinnedCap bytes in
// total, in slabs), and uploads copy from that immutable copy; lookups go
// through a hash index, so a call's cost does not grow with the number of
// distinct tables seen (every streaming append has a plan of its own).  Outside capture a table
// that does not fit any more is copied from the caller's memory, and the call
// waits for that copy;
// under capture (where allocating is not allowed) a table that was never
// uploaded outside capture is an error, so one eager call with the same
// arguments must precede the capture.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>
#include <unordered_map>

#include "skmp_common.hpp"

namespace skmp {

namespace {
struct Blob {
  uint64_t hash;
  size_t bytes;
  void* host;
};
constexpr size_t kPinnedCap = size_t(64) << 20;
// Pinned memory comes in slabs and tables are placed one after the other
// (256-byte aligned), so caching a new table costs a memcpy, not a pinned
// allocation; a table larger than a slab gets its own allocation.
constexpr size_t kSlab = size_t(1) << 20;
std::mutex g_mu;
std::unordered_multimap<uint64_t, Blob> g_blobs;  // by content hash
char* g_slab = nullptr;
size_t g_slab_used = kSlab;
size_t g_total = 0;  // pinned bytes allocated (slabs and large tables)

// Content hash of a table, 8 bytes per step (a match is confirmed with memcmp,
// so the hash only has to separate tables quickly).
uint64_t table_hash(const void* p, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  uint64_t h = 0x9E3779B97F4A7C15ull ^ n;
  size_t i = 0;
  for (; i + 8 <= n; i += 8) {
    uint64_t w;
    memcpy(&w, c + i, 8);
    h = (h ^ (w * 0xBF58476D1CE4E5B9ull)) * 0x94D049BB133111EBull;
    h ^= h >> 31;
  }
  for (; i < n; ++i) h = (h ^ c[i]) * 0x100000001B3ull;
  return h;
}

const Blob* find_blob(uint64_t h, const void* src, size_t bytes) {
  auto range = g_blobs.equal_range(h);
  for (auto it = range.first; it != range.second; ++it)
    if (it->second.bytes == bytes && memcmp(it->second.host, src, bytes) == 0) return &it->second;
  return nullptr;
}

// Pinned space for a new table, nullptr when the cap is reached.
void* pinned_space(size_t bytes) {
  const size_t need = (bytes + 255) & ~size_t(255);
  if (need > kSlab / 4) {  // large: its own allocation
    if (g_total + need > kPinnedCap) return nullptr;
    void* p = nullptr;
    if (hipHostMalloc(&p, need, hipHostMallocDefault) != hipSuccess) return nullptr;
    g_total += need;
    return p;
  }
  if (g_slab_used + need > kSlab) {
    if (g_total + kSlab > kPinnedCap) return nullptr;
    void* p = nullptr;
    if (hipHostMalloc(&p, kSlab, hipHostMallocDefault) != hipSuccess) return nullptr;
    g_slab = static_cast<char*>(p);
    g_slab_used = 0;
    g_total += kSlab;
  }
  void* p = g_slab + g_slab_used;
  g_slab_used += need;
  return p;
}
}  // namespace

bool stream_capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) return false;
  return cs != hipStreamCaptureStatusNone;
}

int upload_async(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return SKMP_OK;
  const bool capturing = stream_capturing(st);
  const uint64_t h = table_hash(src, bytes);
  std::lock_guard<std::mutex> lk(g_mu);
  const Blob* hit = find_blob(h, src, bytes);
  if (!hit && !capturing) {
    if (void* p = pinned_space(bytes)) {
      memcpy(p, src, bytes);
      hit = &g_blobs.emplace(h, Blob{h, bytes, p})->second;
    }
  }
  if (hit) {
    SKMP_CHECK_HIP(hipMemcpyAsync(dst, hit->host, bytes, hipMemcpyHostToDevice, st));
    return SKMP_OK;
  }
  if (capturing) {
    set_error("graph capture: this call's host tables were never uploaded outside capture; make one call with the "
              "same arguments before capturing");
    return SKMP_EINVAL;
  }
  // Past the pinned cap: the source may be a temporary of the calling entry
  // point, so the copy is enqueued in stream order and waited for before the
  // call returns (only tables beyond 64 MiB of distinct content take this path).
  SKMP_CHECK_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
  SKMP_CHECK_HIP(hipStreamSynchronize(st));
  return SKMP_OK;
}

}  // namespace skmp
