// noalloc.hip -- rst_components_noalloc: component labels (Sec. III-B hooking
// and pointer jumping) without any device allocation, for callers that cannot
// allocate (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc).  The hooking runs the global sweep of ghook.hip; its only
// scratch (the recorded edge of every slot, which the sweep writes, and the
// counters) lives in one file-scope device array of fixed size, so the call
// allocates nothing.  Every GPU the library runs on holds its own copy of the
// array until the process ends; all calls on one GPU share it, so calls that
// overlap on one GPU race.
#include "rst_internal.h"

namespace rst {

// scratch: kNoallocCounterBytes of counters, then tu[n] and tv[n]
constexpr size_t kNoallocCounterBytes = 256;
constexpr size_t kNoallocBytes = (size_t)128 << 20;   // 128 MiB per GPU

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

// Device address of `scratch` per device (the array's name in host code is a
// host-side stand-in, not a device address).
constexpr int kNoallocMaxDevices = 64;
static void *g_scratch_dev[kNoallocMaxDevices] = {};

rst_status noalloc_init(int device) {
  if (device < 0 || device >= kNoallocMaxDevices) return RST_OK;   // entry point then refuses
  if (g_scratch_dev[device]) return RST_OK;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return RST_E_DEVICE;
  }
  g_scratch_dev[device] = p;
  return RST_OK;
}

int64_t noalloc_max_vertices() {
  return (int64_t)((kNoallocBytes - kNoallocCounterBytes) / (2 * sizeof(int32_t)));
}

}  // namespace rst

using namespace rst;

extern "C" rst_status rst_components_noalloc(rst_ctx *ctx, const rst_csr *g, int32_t *label,
                                             int64_t *num_components) {
  if (!ctx || !label || !g || g->n < 1 || !g->offsets) return RST_E_INVAL;
  if (g->nnz < 0 || (g->nnz > 0 && !g->cols)) return RST_E_INVAL;
  if (g->offset_bytes != 4 && g->offset_bytes != 8) return RST_E_INVAL;
  // the sweep's per-workgroup arc counts are int32; the scratch holds tu, tv
  if (g->nnz >= ((int64_t)1 << 31) || g->n > noalloc_max_vertices()) return RST_E_INVAL;
  if (ctx->device < 0 || ctx->device >= kNoallocMaxDevices || !g_scratch_dev[ctx->device])
    return RST_E_DEVICE;
  RST_HIP(hipSetDevice(ctx->device));
  char *base = static_cast<char *>(g_scratch_dev[ctx->device]);
  ForestBufs f;
  f.counters = reinterpret_cast<int32_t *>(base);
  f.tu = reinterpret_cast<int32_t *>(base + kNoallocCounterBytes);
  f.tv = f.tu + g->n;
  f.cc = label;
  f.head = nullptr;   // labels only: no Euler arc lists
  // counters start from zero (a fill kernel: no memset node if captured)
  RST_TRY(enqueue_fill(ctx, f.counters, (int64_t)(kNoallocCounterBytes / 4), 0));
  RST_TRY(enqueue_hook_global(ctx, g, f));
  RST_TRY(enqueue_compress(ctx, g->n, label, nullptr, nullptr));
  RST_TRY(enqueue_count_roots(ctx, g->n, label, f.counters));
  RST_HIP(hipMemcpyAsync(ctx->host_pinned, f.counters, kCntTotal * sizeof(int32_t),
                         hipMemcpyDeviceToHost, ctx->stream));
  RST_HIP(hipStreamSynchronize(ctx->stream));
  if (num_components) *num_components = ctx->host_pinned[kCntComponents];
  return RST_OK;
}
