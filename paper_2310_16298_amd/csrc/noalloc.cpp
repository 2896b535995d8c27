// stencil_run_steps_noalloc: the steps of stencil_run_steps for callers that
// cannot allocate device memory.  The plan's operands (band fragments, dense
// C^g, zero line) live in a static device array instead of the three
// allocations a plan object makes.
//
// Host code never uses the array's name as an address: in host code it names
// a host-side stand-in, and a kernel handed that would fault.  The device
// address is looked up once per device with hipGetSymbolAddress (with that
// device current) and kept; kernel arguments are derived from it.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "runtime.hpp"

using namespace stencil;

namespace {

constexpr size_t kScratchBytes = STENCIL_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

}  // namespace

// The operands of the last call on this device; shared by every call.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {nullptr};

// Device address of `scratch` on the current device, looked up on first use.
stencil_status_t scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return STENCIL_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return STENCIL_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return STENCIL_EHIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return STENCIL_OK;
}

// A piece of the operand image carried in the kernel arguments (kernarg
// segment: copied at launch, so the host bytes may go away right after).
constexpr int kPieceWords = 760;
struct ScratchPiece {
  uint32_t offset;  // byte offset into the array, a multiple of 4
  uint32_t words;   // 32-bit words in data
  uint32_t data[kPieceWords];
};

__global__ __launch_bounds__(256) void scratch_fill(unsigned char* base, ScratchPiece p) {
  uint32_t* dst = reinterpret_cast<uint32_t*>(base + p.offset);
  for (uint32_t i = threadIdx.x; i < p.words; i += blockDim.x) dst[i] = p.data[i];
}

// Write `image` (a multiple of 4 bytes) to base on `s`.
stencil_status_t upload(unsigned char* base, const std::vector<uint8_t>& image, hipStream_t s) {
  ScratchPiece p;
  for (size_t off = 0; off < image.size(); off += sizeof(p.data)) {
    const size_t n = std::min(sizeof(p.data), image.size() - off);
    p.offset = (uint32_t)off;
    p.words = (uint32_t)(n / 4);
    std::memcpy(p.data, image.data() + off, n);
    void* args[] = {&base, &p};
    if (hipLaunchKernel(reinterpret_cast<const void*>(scratch_fill), dim3(1), dim3(256), args, 0, s) != hipSuccess)
      return STENCIL_EHIP;
  }
  return STENCIL_OK;
}

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

extern "C" stencil_status_t stencil_run_steps_noalloc(const stencil_desc_t* desc, void* buf0, void* buf1,
                                                      int64_t steps, void* stream, int32_t* result_index) {
  if (!desc || !buf0 || !buf1 || steps < 0) return STENCIL_EINVAL;
  try {
    Resolved rs;
    const int st = resolve_plan(desc, &rs, true);
    if (st != STENCIL_OK) return (stencil_status_t)st;
    if (overlaps(buf0, buf1, grid_bytes_of(desc))) return STENCIL_EALIAS;
    // image: zero line, dense C^g, fragments (each at a 256-byte boundary)
    const size_t coef_off = 256, frag_off = coef_off + up256(rs.coef.size());
    const size_t total = frag_off + up256(rs.frag.size());
    if (total != (size_t)rs.info.operand_bytes || total > kScratchBytes) return STENCIL_ETOOBIG;
    if (result_index) *result_index = 0;
    if (steps == 0) return STENCIL_OK;

    hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return STENCIL_EHIP;
    if (cs != hipStreamCaptureStatusNone) return STENCIL_EUNSUPPORTED;
    void* base = nullptr;
    const stencil_status_t sa = scratch_address(&base);
    if (sa != STENCIL_OK) return sa;

    std::vector<uint8_t> image(total, 0);
    if (!rs.coef.empty()) std::memcpy(image.data() + coef_off, rs.coef.data(), rs.coef.size());
    if (!rs.frag.empty()) std::memcpy(image.data() + frag_off, rs.frag.data(), rs.frag.size());
    unsigned char* b = static_cast<unsigned char*>(base);
    const stencil_status_t su = upload(b, image, s);
    if (su != STENCIL_OK) return su;
    rs.args.zeros = b;
    rs.args.coef = b + coef_off;
    rs.args.frag = rs.frag.empty() ? nullptr : b + frag_off;

    const stencil_status_t sl = launch_steps(rs, buf0, buf1, steps, s);
    if (sl != STENCIL_OK) return sl;
    if (result_index) *result_index = (int32_t)(launch_count(rs, steps) & 1);
    return STENCIL_OK;
  } catch (...) {
    return STENCIL_EINTERNAL;
  }
}
