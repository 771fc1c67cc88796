// Context, workspace and error plumbing.
#include "internal.hpp"

namespace bkts {

static thread_local std::string g_last_error;

std::string fmt(const char* f, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, f);
  vsnprintf(buf, sizeof buf, f, ap);
  va_end(ap);
  return std::string(buf);
}

void set_last_error(const std::string& m) { g_last_error = m; }
const char* last_error() { return g_last_error.c_str(); }

void DevBuf::alloc(size_t n) {
  release();
  if (n == 0) return;
  hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) {
    p = nullptr;
    throw Error{BKTS_ENOMEM, fmt("hipMalloc(%zu bytes) failed: %s", n, hipGetErrorString(e))};
  }
  bytes = n;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

void* Workspace::get(const std::string& name, size_t bytes) {
  DevBuf& b = bufs[name];
  if (b.bytes < bytes) {
    // grow with headroom so that alternating sizes do not reallocate every call
    size_t want = bytes + bytes / 8 + 256;
    b.alloc(want);
  }
  return b.p;
}

size_t Workspace::total_bytes() const {
  size_t s = 0;
  for (auto& kv : bufs) s += kv.second.bytes;
  return s;
}

hipEvent_t Profiler::take() {
  if (pool.empty()) {
    hipEvent_t e;
    // timing only: no system-scope fence on completion, so a timed kernel is not charged for an L2
    // write-back of what earlier kernels left dirty, and the next kernel does not pay for it either
    BKTS_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    return e;
  }
  hipEvent_t e = pool.back();
  pool.pop_back();
  return e;
}

void Profiler::resolve() {
  for (auto& r : pending) {
    BKTS_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    BKTS_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    acc[r.kid].ms += ms;
    acc[r.kid].samples.push_back(ms);
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  pending.clear();
}

void Profiler::reset() {
  for (auto& a : acc) a = Acc{};
  for (auto& s : seq) s = 0;
}

Profiler::~Profiler() {
  for (auto& r : pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

ProfScope::ProfScope(bkts_ctx c, int k, double bytes) : ctx(c), kid(k) {
  if (!ctx->prof.enabled) return;
  Profiler& p = ctx->prof;
  if (p.seq[k]++ % p.period != 0) return;  // not a sampled launch
  if (p.pending.size() > 8192 && p.open == 0) p.resolve();  // only when every event is recorded
  if (p.ext_a) {  // an enclosing scope has not launched its kernel: record its events as empty
    BKTS_HIP(hipEventRecord(p.ext_a, ctx->stream));
    BKTS_HIP(hipEventRecord(p.ext_b, ctx->stream));
    p.ext_a = p.ext_b = nullptr;
    p.open -= 1;
  }
  a = p.take();
  b = p.take();
  p.pending.push_back({k, a, b});
  p.acc[k].launches += 1;
  p.acc[k].bytes += bytes;
  p.ext_a = a;
  p.ext_b = b;
  p.open += 1;
}

void ProfScope::end() {
  if (!a) return;
  Profiler& p = ctx->prof;
  if (p.ext_a == a) {  // no kernel was launched in the scope
    (void)hipEventRecord(a, ctx->stream);
    (void)hipEventRecord(b, ctx->stream);
    p.ext_a = p.ext_b = nullptr;
    p.open -= 1;
  }
  a = b = nullptr;
}

int blocks_per_cu(const void* kernel) {
  static thread_local std::map<const void*, int> cache;
  auto it = cache.find(kernel);
  if (it != cache.end()) return it->second;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, 256, 0) != hipSuccess || n < 1) n = 2;
  cache[kernel] = n;
  return n;
}

}  // namespace bkts

unsigned* bkts_ctx_s::tail_counter(int i) {
  constexpr int kCounters = 16;
  if (!tail_counters.p) {
    tail_counters.alloc(sizeof(unsigned) * kCounters);
    BKTS_HIP(hipMemsetAsync(tail_counters.p, 0, sizeof(unsigned) * kCounters, stream));
  }
  return tail_counters.as<unsigned>() + (i % kCounters);
}

double* bkts_ctx_s::host_stage(size_t count) {
  size_t bytes = count * sizeof(double);
  if (h_pinned_bytes < bytes) {
    if (h_pinned) (void)hipHostFree(h_pinned);
    h_pinned = nullptr;
    h_pinned_bytes = 0;
    size_t want = bytes < 65536 ? 65536 : bytes;
    // coherent: kernels may write results straight into it (the fused block-CG tail does)
    BKTS_HIP(hipHostMalloc(reinterpret_cast<void**>(&h_pinned), want, hipHostMallocCoherent));
    h_pinned_bytes = want;
  }
  return h_pinned;
}

void bkts_ctx_s::sync() { BKTS_HIP(hipStreamSynchronize(stream)); }
