// C ABI of the library (see include/ffbspca.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>

#include "../../include/ffbspca.h"
#include "kernels.h"
#include "plan.h"

namespace {

constexpr int64_t kMaxPassImages = 16384;  // gridDim.y of the per-image kernels stays far below 65535
constexpr size_t kAlign = 256;             // both pass buffers start on 256-byte boundaries

int64_t round_group(int64_t m) { return (m + fb::kImgGroup - 1) / fb::kImgGroup * fb::kImgGroup; }

// Images per pass that fit the workspace, and the two pass buffers inside it.  A pass
// of nb images uses round_group(nb) image slots in each buffer.
int64_t split_workspace(const fb::PassLayout& lay, void* ws, size_t ws_bytes, int64_t n, float2** a, float2** b) {
  uintptr_t base = ((uintptr_t)ws + kAlign - 1) & ~(uintptr_t)(kAlign - 1);
  size_t skip = base - (uintptr_t)ws;
  if (ws_bytes < skip + kAlign) return 0;
  size_t avail = ws_bytes - skip - kAlign;
  int64_t slots = (int64_t)(avail / lay.per_image) / fb::kImgGroup * fb::kImgGroup;
  int64_t nb = std::min<int64_t>({n, slots, kMaxPassImages});
  if (nb < 1) return 0;
  // The pass buffers keep images innermost with a row stride of nb images.  A stride
  // that is a multiple of 2 KiB puts every row of a workgroup's tile on the same HBM
  // channels; 16 images fewer (still a whole 128-byte line) spreads them.
  if (nb >= 512 && nb % 256 == 0) nb -= 16;
  *a = (float2*)base;
  size_t off_b = (lay.bytes_a * (size_t)round_group(nb) + kAlign - 1) & ~(kAlign - 1);
  *b = (float2*)(base + off_b);
  return nb;
}

int make_plan(int L, double c, double R, bool device, fb_plan_t* out) {
  if (!out) return FB_ERR_INVALID_ARG;
  *out = nullptr;
  fb_plan_s* h = new (std::nothrow) fb_plan_s();
  if (!h) return FB_ERR_ALLOC;
  int rc;
  try {
    rc = fb::build_host_plan(L, c, R, h->pl);
  } catch (const std::bad_alloc&) {
    rc = FB_ERR_ALLOC;
  } catch (...) {
    rc = FB_ERR_INVALID_ARG;
  }
  if (rc == FB_OK && device) rc = fb::upload_plan(h->pl);
  if (rc != FB_OK) {
    fb::free_device(h->pl);
    delete h;
    return rc;
  }
  *out = h;
  return FB_OK;
}

int hip_rc(fb::Plan& pl, hipError_t e) {
  if (e == hipSuccess) return FB_OK;
  pl.last_hip = e;
  return FB_ERR_HIP;
}

}  // namespace

extern "C" {

int fb_plan(int L, double c, double R, fb_plan_t* out) { return make_plan(L, c, R, true, out); }

int fb_plan_host(int L, double c, double R, fb_plan_t* out) { return make_plan(L, c, R, false, out); }

int fb_plan_destroy(fb_plan_t plan) {
  if (!plan) return FB_OK;
  fb::free_device(plan->pl);
  delete plan;
  return FB_OK;
}

int fb_plan_info(fb_plan_t plan, fb_info* out) {
  if (!plan || !out) return FB_ERR_INVALID_ARG;
  const fb::Plan& p = plan->pl;
  out->L = p.L;
  out->c = p.c;
  out->R = p.R;
  out->n_xi = p.n_xi;
  out->n_theta = p.n_theta;
  out->k_max = p.k_max;
  out->p0 = p.p0;
  out->p_half = p.p_half;
  out->p_total = p.p_total;
  out->cov_size = p.cov_size;
  out->grid_n = p.N;
  out->kernel_w = p.w;
  out->kernel_beta = p.beta;
  out->has_device = p.has_device ? 1 : 0;
  return FB_OK;
}

int fb_plan_tables(fb_plan_t plan, int32_t* k, int32_t* q, int32_t* p, int64_t* coef_off, int64_t* cov_off) {
  if (!plan) return FB_ERR_INVALID_ARG;
  const fb::Plan& pl = plan->pl;
  if (k) std::copy(pl.kq_k.begin(), pl.kq_k.end(), k);
  if (q) std::copy(pl.kq_q.begin(), pl.kq_q.end(), q);
  if (p) std::copy(pl.p.begin(), pl.p.end(), p);
  if (coef_off) std::copy(pl.coef_off.begin(), pl.coef_off.end(), coef_off);
  if (cov_off) std::copy(pl.cov_off.begin(), pl.cov_off.end(), cov_off);
  return FB_OK;
}

int fb_plan_host_tables(fb_plan_t plan, double* roots, double* norms, double* xi, double* w, double* radial) {
  if (!plan) return FB_ERR_INVALID_ARG;
  const fb::Plan& pl = plan->pl;
  if (roots) std::copy(pl.roots.begin(), pl.roots.end(), roots);
  if (norms) std::copy(pl.norms.begin(), pl.norms.end(), norms);
  if (xi) std::copy(pl.xi.begin(), pl.xi.end(), xi);
  if (w) std::copy(pl.wq.begin(), pl.wq.end(), w);
  if (radial) std::copy(pl.radial.begin(), pl.radial.end(), radial);
  return FB_OK;
}

size_t fb_workspace_bytes(fb_plan_t plan, int64_t batch, int precision) {
  (void)precision;
  if (!plan || batch < 1) return 0;
  return fb::pass_layout(plan->pl).per_image * (size_t)round_group(std::min<int64_t>(batch, kMaxPassImages)) + kAlign;
}

int fb_expand(fb_plan_t plan, const float* images, int64_t n, float* coeffs, int precision, void* ws,
              size_t ws_bytes, void* stream) {
  return fb_expand_weighted(plan, images, n, coeffs, precision, 1, ws, ws_bytes, stream);
}

int fb_expand_weighted(fb_plan_t plan, const float* images, int64_t n, float* coeffs, int precision,
                       int weight_mode, void* ws, size_t ws_bytes, void* stream) {
  if (!plan || n < 0 || (weight_mode != 0 && weight_mode != 1)) return FB_ERR_INVALID_ARG;
  if (precision != FB_FP32 && precision != FB_BF16X3) return FB_ERR_INVALID_ARG;
  if (n == 0) return FB_OK;
  if (!images || !coeffs || !ws) return FB_ERR_INVALID_ARG;
  fb::Plan& pl = plan->pl;
  if (!pl.has_device) return FB_ERR_NO_DEVICE;
  fb::PassLayout lay = fb::pass_layout(pl);
  float2 *bufA = nullptr, *bufB = nullptr;
  int64_t nb = split_workspace(lay, ws, ws_bytes, n, &bufA, &bufB);
  if (nb < 1) return FB_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  const size_t img_stride = (size_t)pl.L * pl.L;
  const size_t coef_stride = 2 * (size_t)pl.p_half;
  for (int64_t s = 0; s < n; s += nb) {
    int m = (int)std::min<int64_t>(nb, n - s);
    int rc = hip_rc(pl, fb::launch_forward_nufft(pl, images + s * img_stride, m, bufA, bufB, st));
    if (rc == FB_OK) rc = hip_rc(pl, fb::launch_forward_angular(pl, bufA, bufB, m, st));
    if (rc == FB_OK)
      rc = hip_rc(pl, fb::launch_radial_forward(pl, bufB, coeffs + s * coef_stride, m, precision, weight_mode, st));
    if (rc != FB_OK) return rc;
  }
  return FB_OK;
}

int fb_adjoint(fb_plan_t plan, const float* coeffs, int64_t n, float* images, int weight_mode, void* ws,
               size_t ws_bytes, void* stream) {
  return fb_adjoint_filtered(plan, coeffs, n, images, weight_mode, nullptr, ws, ws_bytes, stream);
}

int fb_adjoint_filtered(fb_plan_t plan, const float* coeffs, int64_t n, float* images, int weight_mode,
                        const float* ring_filter, void* ws, size_t ws_bytes, void* stream) {
  if (!plan || n < 0 || (weight_mode != 0 && weight_mode != 1)) return FB_ERR_INVALID_ARG;
  if (n == 0) return FB_OK;
  if (!images || !coeffs || !ws) return FB_ERR_INVALID_ARG;
  fb::Plan& pl = plan->pl;
  if (!pl.has_device) return FB_ERR_NO_DEVICE;
  fb::PassLayout lay = fb::pass_layout(pl);
  float2 *bufA = nullptr, *bufB = nullptr;
  int64_t nb = split_workspace(lay, ws, ws_bytes, n, &bufA, &bufB);
  if (nb < 1) return FB_ERR_WORKSPACE;
  nb = std::min(nb, fb::spread_max_images(pl));
  hipStream_t st = (hipStream_t)stream;
  const size_t img_stride = (size_t)pl.L * pl.L;
  const size_t coef_stride = 2 * (size_t)pl.p_half;
  for (int64_t s = 0; s < n; s += nb) {
    int m = (int)std::min<int64_t>(nb, n - s);
    int rc = hip_rc(pl, fb::launch_radial_adjoint(pl, coeffs + s * coef_stride, bufB, m, weight_mode,
                                                  ring_filter, st));
    if (rc == FB_OK) rc = hip_rc(pl, fb::launch_adjoint_angular(pl, bufB, bufA, m, st));
    if (rc == FB_OK) rc = hip_rc(pl, fb::launch_adjoint_nufft(pl, bufA, m, bufA, bufB, images + s * img_stride, st));
    if (rc != FB_OK) return rc;
  }
  return FB_OK;
}

size_t fb_covariance_workspace_bytes(fb_plan_t plan, int64_t n, int hermitian) {
  if (!plan || n <= 0) return 0;
  return fb::cov_split(plan->pl, n, hermitian != 0).bytes;
}

int fb_covariance_shift(fb_plan_t plan, const float* coeffs, int64_t n, float* shift, void* stream) {
  if (!plan || n <= 0 || !coeffs || !shift) return FB_ERR_INVALID_ARG;
  fb::Plan& pl = plan->pl;
  if (!pl.has_device) return FB_ERR_NO_DEVICE;
  return hip_rc(pl, fb::launch_cov_shift(pl, coeffs, n, shift, (hipStream_t)stream));
}

int fb_covariance(fb_plan_t plan, const float* coeffs, int64_t n, double* G, double* S0, double* Gi,
                  const float* shift, int64_t* count, int precision, void* ws, size_t ws_bytes, void* stream) {
  if (!plan || n < 0) return FB_ERR_INVALID_ARG;
  if (precision != FB_FP32 && precision != FB_BF16X3) return FB_ERR_INVALID_ARG;
  if (!G || !S0 || !count || *count < 0) return FB_ERR_INVALID_ARG;
  fb::Plan& pl = plan->pl;
  if (!pl.has_device) return FB_ERR_NO_DEVICE;
  if (n == 0) return FB_OK;
  if (!coeffs || !ws || ((uintptr_t)ws & 7)) return FB_ERR_INVALID_ARG;
  if (ws_bytes < fb::cov_split(pl, n, Gi != nullptr).bytes) return FB_ERR_WORKSPACE;
  int rc = hip_rc(pl, fb::launch_covariance(pl, coeffs, n, G, S0, Gi, shift, precision, ws, (hipStream_t)stream));
  if (rc == FB_OK) *count += n;
  return rc;
}

size_t fb_eig_workspace_bytes(fb_plan_t plan) { return plan ? fb::eig_workspace_bytes(plan->pl) : 0; }

int fb_eig(fb_plan_t plan, const double* G, const double* S0, const float* shift, int64_t count, double* evals,
           double* evecs, double* C_out, double* mean_out, void* ws, size_t ws_bytes, void* stream) {
  if (!plan || count <= 0 || !G || !S0 || !evals || !evecs || !ws) return FB_ERR_INVALID_ARG;
  fb::Plan& pl = plan->pl;
  if (!pl.has_device) return FB_ERR_NO_DEVICE;
  if (ws_bytes < fb::eig_workspace_bytes(pl)) return FB_ERR_WORKSPACE;
  return hip_rc(pl, fb::launch_eig(pl, G, S0, shift, count, evals, evecs, C_out, mean_out, (double*)ws,
                                   (hipStream_t)stream));
}

int fb_spca_select(fb_plan_t plan, const double* evals, int64_t count, double sigma2, int32_t* n_sel,
                   double* weights, void* stream) {
  if (!plan || !evals || !n_sel || !weights || count <= 0 || !(sigma2 >= 0.0)) return FB_ERR_INVALID_ARG;
  fb::Plan& pl = plan->pl;
  if (!pl.has_device) return FB_ERR_NO_DEVICE;
  return hip_rc(pl, fb::launch_spca_select(pl, evals, count, sigma2, n_sel, weights, (hipStream_t)stream));
}

int fb_spca_coeffs(fb_plan_t plan, const float* coeffs, int64_t n, const double* evecs, const double* mean,
                   float* out, void* stream) {
  if (!plan || n < 0) return FB_ERR_INVALID_ARG;
  fb::Plan& pl = plan->pl;
  if (!pl.has_device) return FB_ERR_NO_DEVICE;
  if (n == 0) return FB_OK;
  if (!coeffs || !evecs || !mean || !out || (const void*)coeffs == (const void*)out) return FB_ERR_INVALID_ARG;
  return hip_rc(pl, fb::launch_spca_apply(pl, 0, coeffs, n, evecs, mean, nullptr, out, (hipStream_t)stream));
}

int fb_spca_reconstruct(fb_plan_t plan, const float* c, int64_t n, const double* evecs, const double* mean,
                        const double* weights, float* out, void* stream) {
  if (!plan || n < 0) return FB_ERR_INVALID_ARG;
  fb::Plan& pl = plan->pl;
  if (!pl.has_device) return FB_ERR_NO_DEVICE;
  if (n == 0) return FB_OK;
  if (!c || !evecs || !mean || !out || (const void*)c == (const void*)out) return FB_ERR_INVALID_ARG;
  return hip_rc(pl, fb::launch_spca_apply(pl, 1, c, n, evecs, mean, weights, out, (hipStream_t)stream));
}

int fb_spca_radial(fb_plan_t plan, const double* evecs, float* f, void* stream) {
  if (!plan || !evecs || !f) return FB_ERR_INVALID_ARG;
  fb::Plan& pl = plan->pl;
  if (!pl.has_device) return FB_ERR_NO_DEVICE;
  return hip_rc(pl, fb::launch_spca_radial(pl, evecs, f, (hipStream_t)stream));
}

size_t fb_moments_workspace_bytes(fb_plan_t plan) {
  if (!plan) return 0;
  return fb::moments_workspace_bytes(plan->pl);
}

int fb_pixel_moments(fb_plan_t plan, const float* images, int64_t n, double* sum, double* sumsq, void* ws,
                     size_t ws_bytes, void* stream) {
  if (!plan || n < 0) return FB_ERR_INVALID_ARG;
  fb::Plan& pl = plan->pl;
  if (!pl.has_device) return FB_ERR_NO_DEVICE;
  if (n == 0) return FB_OK;
  if (!images || !sum || !sumsq || !ws || (uintptr_t)ws % 8 != 0) return FB_ERR_INVALID_ARG;
  if (ws_bytes < fb::moments_workspace_bytes(pl)) return FB_ERR_WORKSPACE;
  return hip_rc(pl, fb::launch_pixel_moments(pl, images, n, sum, sumsq, (double*)ws, (hipStream_t)stream));
}

// polar power workspace: mean image (L^2 floats), its polar samples (n_xi H complex), then
// the pass buffers of fb_expand
static size_t power_head_bytes(const fb::Plan& pl) {
  const size_t a = ((size_t)pl.L * pl.L * sizeof(float) + kAlign - 1) & ~(size_t)(kAlign - 1);
  const size_t b = ((size_t)pl.n_xi * pl.H * sizeof(float2) + kAlign - 1) & ~(size_t)(kAlign - 1);
  return a + b + kAlign;
}

size_t fb_polar_power_workspace_bytes(fb_plan_t plan, int64_t batch) {
  if (!plan || batch < 1) return 0;
  return power_head_bytes(plan->pl) + fb_workspace_bytes(plan, batch, FB_FP32);
}

int fb_polar_power(fb_plan_t plan, const float* images, int64_t n, const double* pixel_sum, int64_t count,
                   double* power, void* ws, size_t ws_bytes, void* stream) {
  if (!plan || n < 0) return FB_ERR_INVALID_ARG;
  fb::Plan& pl = plan->pl;
  if (!pl.has_device) return FB_ERR_NO_DEVICE;
  if (n == 0) return FB_OK;
  if (!images || !power || !ws || (pixel_sum && count <= 0)) return FB_ERR_INVALID_ARG;
  const size_t head = power_head_bytes(pl);
  if (ws_bytes < head) return FB_ERR_WORKSPACE;
  const uintptr_t base = ((uintptr_t)ws + kAlign - 1) & ~(uintptr_t)(kAlign - 1);
  float* mean = (float*)base;
  float2* pmean = (float2*)(base + (((size_t)pl.L * pl.L * sizeof(float) + kAlign - 1) & ~(size_t)(kAlign - 1)));
  void* rest = (char*)ws + head;
  fb::PassLayout lay = fb::pass_layout(pl);
  float2 *bufA = nullptr, *bufB = nullptr;
  int64_t nb = split_workspace(lay, rest, ws_bytes - head, n, &bufA, &bufB);
  if (nb < 1) return FB_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  int rc = FB_OK;
  if (pixel_sum) {
    rc = hip_rc(pl, fb::launch_mean_image(pl, pixel_sum, count, mean, st));
    if (rc == FB_OK) rc = hip_rc(pl, fb::launch_forward_nufft(pl, mean, 1, bufA, bufB, st));
    if (rc == FB_OK) rc = hip_rc(pl, fb::launch_copy_polar(pl, bufA, pmean, st));
    if (rc != FB_OK) return rc;
  }
  const size_t img_stride = (size_t)pl.L * pl.L;
  for (int64_t s = 0; s < n; s += nb) {
    int m = (int)std::min<int64_t>(nb, n - s);
    rc = hip_rc(pl, fb::launch_forward_nufft(pl, images + s * img_stride, m, bufA, bufB, st));
    if (rc == FB_OK) rc = hip_rc(pl, fb::launch_polar_power(pl, bufA, pixel_sum ? pmean : nullptr, m, power, st));
    if (rc != FB_OK) return rc;
  }
  return FB_OK;
}

int fb_estimate_support(fb_plan_t plan, const double* sum, const double* sumsq, int64_t n, const double* power,
                        double noise_var, double frac, double* out, void* stream) {
  if (!plan || n <= 0 || !sum || !sumsq || !power || !out || !(frac > 0.0 && frac <= 1.0)) return FB_ERR_INVALID_ARG;
  fb::Plan& pl = plan->pl;
  if (!pl.has_device) return FB_ERR_NO_DEVICE;
  return hip_rc(pl, fb::launch_estimate_support(pl, sum, sumsq, n, power, noise_var, frac, out, (hipStream_t)stream));
}

int fb_ctf_filter(fb_plan_t plan, double pixel_size, double lambda, double defocus, double phase, double bfactor,
                  float* filter, void* stream) {
  if (!plan || !filter || !(pixel_size > 0.0) || !std::isfinite(pixel_size) || !std::isfinite(lambda) ||
      !std::isfinite(defocus) || !std::isfinite(phase) || !std::isfinite(bfactor))
    return FB_ERR_INVALID_ARG;
  fb::Plan& pl = plan->pl;
  if (!pl.has_device) return FB_ERR_NO_DEVICE;
  return hip_rc(pl, fb::launch_ctf_filter(pl, pixel_size, lambda, defocus, phase, bfactor, filter,
                                          (hipStream_t)stream));
}

size_t fb_svd_workspace_bytes(fb_plan_t plan, int64_t n) {
  if (!plan || n <= 0) return 0;
  return (size_t)fb::svd_split(plan->pl, n).total_doubles * sizeof(double);
}

int fb_svd(fb_plan_t plan, const float* coeffs, int64_t n, double* evals, double* evecs, double* mean_out, void* ws,
           size_t ws_bytes, void* stream) {
  if (!plan || n <= 0 || !coeffs || !evals || !evecs || !ws) return FB_ERR_INVALID_ARG;
  fb::Plan& pl = plan->pl;
  if (!pl.has_device) return FB_ERR_NO_DEVICE;
  if (fb::svd_finish_lds_bytes(pl) > (size_t)fb::kSvdLdsLimit || fb::svd_max_p(pl) > fb::kSvdMaxP)
    return FB_ERR_UNSUPPORTED;
  if ((uintptr_t)ws % 8 != 0) return FB_ERR_INVALID_ARG;
  if (ws_bytes < fb_svd_workspace_bytes(plan, n)) return FB_ERR_WORKSPACE;
  const fb::SvdSplit s = fb::svd_split(pl, n);
  if ((long long)s.W0 + (long long)s.W1 * pl.k_max > 0x7fffffffLL) return FB_ERR_INVALID_ARG;
  return hip_rc(pl, fb::launch_svd(pl, coeffs, n, evals, evecs, mean_out, (double*)ws, (hipStream_t)stream));
}

int fb_eigenimages(fb_plan_t plan, const double* evecs, int k, int l0, int nl, double* out, void* stream) {
  if (!plan || nl < 0 || l0 < 0) return FB_ERR_INVALID_ARG;
  fb::Plan& pl = plan->pl;
  if (!pl.has_device) return FB_ERR_NO_DEVICE;
  if (k < 0 || k > pl.k_max || l0 + nl > pl.p[k]) return FB_ERR_INVALID_ARG;
  if (nl == 0) return FB_OK;
  if (!evecs || !out) return FB_ERR_INVALID_ARG;
  return hip_rc(pl, fb::launch_eigenimages(pl, evecs, k, l0, nl, out, (hipStream_t)stream));
}

int fb_synth_normals(uint64_t seed, uint32_t rng_stream, int64_t first_index, int64_t n, int64_t n_per, float scale,
                     float* out, void* stream) {
  if (n < 0 || n_per < 0 || first_index < 0) return FB_ERR_INVALID_ARG;
  if (n == 0 || n_per == 0) return FB_OK;
  if (!out) return FB_ERR_INVALID_ARG;
  return fb::launch_synth_normals(seed, rng_stream, first_index, n, n_per, scale, out, (hipStream_t)stream) ==
                 hipSuccess
             ? FB_OK
             : FB_ERR_HIP;
}

int fb_synth_words(uint64_t seed, uint32_t rng_stream, int64_t first_index, int64_t n, int64_t n_per, uint32_t* out,
                   void* stream) {
  if (n < 0 || n_per < 0 || first_index < 0) return FB_ERR_INVALID_ARG;
  if (n == 0 || n_per == 0) return FB_OK;
  if (!out) return FB_ERR_INVALID_ARG;
  return fb::launch_synth_words(seed, rng_stream, first_index, n, n_per, out, (hipStream_t)stream) == hipSuccess
             ? FB_OK
             : FB_ERR_HIP;
}

int fb_profile_enable(fb_plan_t plan, int enable) {
  if (!plan) return FB_ERR_INVALID_ARG;
  if (!plan->pl.has_device) return FB_ERR_NO_DEVICE;
  plan->pl.prof.on = enable != 0;
  return FB_OK;
}

int fb_profile_read(fb_plan_t plan, double* total_ms, int64_t* launches, int max_stages, int reset) {
  if (!plan || max_stages < 0) return FB_ERR_INVALID_ARG;
  fb::Profiler& pr = plan->pl.prof;
  int rc = pr.collect();
  if (rc != FB_OK) return rc;
  for (int s = 0; s < std::min(max_stages, (int)fb::ST_COUNT); ++s) {
    if (total_ms) total_ms[s] = pr.total_ms[s];
    if (launches) launches[s] = pr.launches[s];
  }
  if (reset)
    for (int s = 0; s < fb::ST_COUNT; ++s) {
      pr.total_ms[s] = 0.0;
      pr.launches[s] = 0;
    }
  return fb::ST_COUNT;
}

const char* fb_stage_name(int stage) { return fb::stage_name(stage); }

const char* fb_error_string(int code) {
  switch (code) {
    case FB_OK: return "success";
    case FB_ERR_INVALID_ARG: return "invalid argument";
    case FB_ERR_ALLOC: return "allocation failed";
    case FB_ERR_HIP: return "HIP runtime error";
    case FB_ERR_UNSUPPORTED: return "unsupported plan parameters";
    case FB_ERR_NO_DEVICE: return "plan has no device tables";
    case FB_ERR_WORKSPACE: return "workspace too small";
    case FB_ERR_SCRATCH_LIMIT: return "one pass of 16 images needs more than the fixed device scratch of fb_expand_noalloc";
    default: return "unknown error";
  }
}

int fb_plan_last_hip_error(fb_plan_t plan) { return plan ? (int)plan->pl.last_hip : 0; }

}  // extern "C"
