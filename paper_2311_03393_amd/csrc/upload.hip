// Host-to-device uploads of small host tables (series plans, sketch
// coefficients) that a HIP graph may capture.
//
// A captured memcpy node reads its host source again at every replay, so the
// source must outlive the graph and never change.  Every uploaded table is
// therefore also kept, once per distinct content, in pinned host memory owned
// by the library for the life of the process (up to kPinnedCap bytes in
// total), and uploads copy from that immutable copy.  Outside capture a table
// that does not fit any more is copied from the caller's memory as before;
// under capture (where allocating is not allowed) a table that was never
// uploaded outside capture is an error, so one eager call with the same
// arguments must precede the capture.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "skmp_common.hpp"

namespace skmp {

namespace {
struct Blob {
  uint64_t hash;
  size_t bytes;
  void* host;
};
constexpr size_t kPinnedCap = size_t(64) << 20;
std::mutex g_mu;
std::vector<Blob> g_blobs;
size_t g_total = 0;

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
  for (const Blob& b : g_blobs)
    if (b.hash == h && b.bytes == bytes && memcmp(b.host, src, bytes) == 0) return &b;
  return nullptr;
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
  if (!hit && !capturing && g_total + bytes <= kPinnedCap) {
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) == hipSuccess && p) {
      memcpy(p, src, bytes);
      g_blobs.push_back({h, bytes, p});
      g_total += bytes;
      hit = &g_blobs.back();
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
  SKMP_CHECK_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
  return SKMP_OK;
}

}  // namespace skmp
