// The extern "C" entry points declared in include/stencil.h.
#include <cstring>
#include <new>

#include "runtime.hpp"

using namespace stencil;

namespace {

void free_plan(stencil_plan_s* p) {
  if (!p) return;
  if (p->d_frag) (void)hipFree(p->d_frag);
  if (p->d_coef) (void)hipFree(p->d_coef);
  if (p->d_zeros) (void)hipFree(p->d_zeros);
  delete p;
}

}  // namespace

extern "C" {

const char* stencil_version(void) { return "paper_2310_16298_amd 0.1.0 (gfx950)"; }

const char* stencil_status_string(stencil_status_t s) {
  // callers may pass any integer: read its bits, not an enum value (a value
  // outside the enumerators is not a valid stencil_status_t in C++)
  int v = 0;
  std::memcpy(&v, &s, sizeof(v) < sizeof(s) ? sizeof(v) : sizeof(s));
  switch (v) {
    case STENCIL_OK: return "ok";
    case STENCIL_EINVAL: return "invalid argument";
    case STENCIL_EUNSUPPORTED: return "unsupported combination";
    case STENCIL_ENOMEM: return "out of memory";
    case STENCIL_EHIP: return "HIP runtime error";
    case STENCIL_EALIAS: return "input and output buffers overlap";
    case STENCIL_EINTERNAL: return "internal error";
    case STENCIL_ETOOBIG: return "plan operands exceed the no-allocation scratch buffer";
  }
  return "unknown status";
}

stencil_status_t stencil_desc_check(const stencil_desc_t* desc) {
  try {
    Resolved rs;
    return (stencil_status_t)resolve_plan(desc, &rs, false);
  } catch (...) {
    return STENCIL_EINTERNAL;
  }
}

stencil_status_t stencil_plan_describe(const stencil_desc_t* desc, stencil_plan_info_t* info) {
  if (!info) return STENCIL_EINVAL;
  try {
    Resolved rs;
    const int st = resolve_plan(desc, &rs, true);
    if (st != STENCIL_OK) return (stencil_status_t)st;
    *info = rs.info;
    return STENCIL_OK;
  } catch (...) {
    return STENCIL_EINTERNAL;
  }
}

stencil_status_t stencil_line_band(const double* coeffs, int32_t radius, int32_t n, int32_t axis,
                                   int32_t index, double* out) {
  if (!coeffs || !out || radius < 1 || radius > 4 || n < 1 || n > 4096 || (axis != 0 && axis != 1) ||
      index < 0 || index > 2 * radius)
    return STENCIL_EINVAL;
  const int K = n + 2 * radius;
  if (axis == 0) {
    for (int p = 0; p < n; ++p)
      for (int x = 0; x < K; ++x) out[(size_t)p * K + x] = band_value(coeffs, radius, n, 0, index, p, x);
  } else {
    for (int y = 0; y < K; ++y)
      for (int q = 0; q < n; ++q) out[(size_t)y * n + q] = band_value(coeffs, radius, n, 1, index, y, q);
  }
  return STENCIL_OK;
}

stencil_status_t stencil_line_cover(const double* coeffs, int32_t radius, int32_t* rows_out, int32_t* cols_out,
                                    int32_t* count) {
  if (!coeffs || !rows_out || !cols_out || radius < 1 || radius > 4) return STENCIL_EINVAL;
  try {
    int r[9], c[9];
    const int n = line_cover(coeffs, radius, r, c);
    for (int k = 0; k < 2 * radius + 1; ++k) {
      rows_out[k] = r[k];
      cols_out[k] = c[k];
    }
    if (count) *count = n;
    return STENCIL_OK;
  } catch (...) {
    return STENCIL_EINTERNAL;
  }
}

stencil_status_t stencil_plan(const stencil_desc_t* desc, stencil_plan_t* out) {
  if (!out) return STENCIL_EINVAL;
  *out = nullptr;
  stencil_plan_s* p = nullptr;
  try {
    p = new (std::nothrow) stencil_plan_s();
    if (!p) return STENCIL_ENOMEM;
    const int st = resolve_plan(desc, &p->rs, true);
    if (st != STENCIL_OK) {
      free_plan(p);
      return (stencil_status_t)st;
    }
    if (hipGetDevice(&p->device) != hipSuccess) {
      free_plan(p);
      return STENCIL_EHIP;
    }
    p->grid_bytes = grid_bytes_of(desc);
    const size_t fb = p->rs.frag.size(), cb = p->rs.coef.size();
    if (fb) {
      if (hipMalloc(&p->d_frag, fb) != hipSuccess) {
        free_plan(p);
        return STENCIL_ENOMEM;
      }
      if (hipMemcpy(p->d_frag, p->rs.frag.data(), fb, hipMemcpyHostToDevice) != hipSuccess) {
        free_plan(p);
        return STENCIL_EHIP;
      }
    }
    if (hipMalloc(&p->d_coef, cb) != hipSuccess) {
      free_plan(p);
      return STENCIL_ENOMEM;
    }
    if (hipMemcpy(p->d_coef, p->rs.coef.data(), cb, hipMemcpyHostToDevice) != hipSuccess) {
      free_plan(p);
      return STENCIL_EHIP;
    }
    if (hipMalloc(&p->d_zeros, 256) != hipSuccess) {
      free_plan(p);
      return STENCIL_ENOMEM;
    }
    static const unsigned char zero_line[256] = {0};
    if (hipMemcpy(p->d_zeros, zero_line, 256, hipMemcpyHostToDevice) != hipSuccess) {
      free_plan(p);
      return STENCIL_EHIP;
    }
    p->rs.args.frag = p->d_frag;
    p->rs.args.coef = p->d_coef;
    p->rs.args.zeros = p->d_zeros;
    *out = p;
    return STENCIL_OK;
  } catch (const std::bad_alloc&) {
    free_plan(p);
    return STENCIL_ENOMEM;
  } catch (...) {
    free_plan(p);
    return STENCIL_EINTERNAL;
  }
}

stencil_status_t stencil_plan_info(stencil_plan_t plan, stencil_plan_info_t* info) {
  if (!plan || !info) return STENCIL_EINVAL;
  *info = plan->rs.info;
  return STENCIL_OK;
}

stencil_status_t stencil_plan_destroy(stencil_plan_t plan) {
  try {
    free_plan(plan);
    return STENCIL_OK;
  } catch (...) {
    return STENCIL_EINTERNAL;
  }
}

stencil_status_t stencil_apply(stencil_plan_t plan, const void* in, void* out, void* stream) {
  if (!plan || !in || !out) return STENCIL_EINVAL;
  if (overlaps(in, out, plan->grid_bytes)) return STENCIL_EALIAS;
  try {
    const stencil_status_t d = check_device(plan->device);
    if (d != STENCIL_OK) return d;
    return launch_one(plan->rs, in, out, (hipStream_t)stream);
  } catch (...) {
    return STENCIL_EINTERNAL;
  }
}

stencil_status_t stencil_run_steps(stencil_plan_t plan, void* buf0, void* buf1, int64_t steps,
                                   void* stream, int32_t* result_index) {
  if (!plan || !buf0 || !buf1 || steps < 0) return STENCIL_EINVAL;
  if (overlaps(buf0, buf1, plan->grid_bytes)) return STENCIL_EALIAS;
  try {
    const stencil_status_t d = check_device(plan->device);
    if (d != STENCIL_OK) return d;
    const stencil_plan_s* p = plan;
    // Runs of a few launches go out directly: a graph replay cost ~7 us more
    // than direct launches of one to ten kernels on MI355X (512^2 FP64, 10
    // steps: 20.9 against 28.5 us), while longer runs of short kernels are
    // bound by the host's launch rate, which the graph lifts.
    constexpr int64_t kDirectLaunches = 4;
    stencil_status_t st = STENCIL_EUNSUPPORTED;
    if (launch_count(plan->rs, steps) > kDirectLaunches)
      st = plan->graphs.run(buf0, buf1, steps, (hipStream_t)stream,
                            [&](hipStream_t cs) { return launch_steps(p->rs, buf0, buf1, steps, cs); });
    if (st == STENCIL_EUNSUPPORTED) st = launch_steps(plan->rs, buf0, buf1, steps, (hipStream_t)stream);
    if (st != STENCIL_OK) return st;
    if (result_index) *result_index = (int32_t)(launch_count(plan->rs, steps) & 1);
    return STENCIL_OK;
  } catch (...) {
    return STENCIL_EINTERNAL;
  }
}

stencil_status_t stencil_error_norms(const void* a, int32_t a_dtype, const double* ref, int64_t n,
                                     double* out, void* stream) {
  if (!a || !ref || !out || n < 0 || (a_dtype != STENCIL_F32 && a_dtype != STENCIL_F64))
    return STENCIL_EINVAL;
  try {
    return launch_error_norms(a, a_dtype, ref, n, out, (hipStream_t)stream) == hipSuccess ? STENCIL_OK
                                                                                          : STENCIL_EHIP;
  } catch (...) {
    return STENCIL_EINTERNAL;
  }
}

}  // extern "C"
