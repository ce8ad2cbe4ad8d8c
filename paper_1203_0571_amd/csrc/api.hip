// Host side of the C ABI declared in include/shape.h: argument checks,
// option conversion and kernel launches on the caller's stream.
#include "kernels.hpp"

using namespace shape;

namespace {

int check_batch(const shape_batch* b) {
  if (!b) return SHAPE_EINVAL;
  if (b->n < 0 || b->n_pixels < 0) return SHAPE_EINVAL;
  if (b->dtype != SHAPE_F32 && b->dtype != SHAPE_F16_SCALED) return SHAPE_EINVAL;
  if (b->n == 0) return SHAPE_OK;
  if (!b->pixels || !b->sigma) return SHAPE_EINVAL;
  if (b->dtype == SHAPE_F16_SCALED && !b->scale) return SHAPE_EINVAL;
  if (!b->side && (b->side0 < kMinSide || b->side0 > kMaxSide)) return SHAPE_EINVAL;
  if (!b->offset && !b->side && b->n > b->n_pixels / ((int64_t)b->side0 * b->side0))
    return SHAPE_EINVAL;  // a uniform batch must fit in the pixel buffer
  return SHAPE_OK;
}

int check_opts(const shape_opts* o) {
  if (!o) return SHAPE_EINVAL;
  if (o->max_iter_centroid < 0 || o->max_iter_moments < 0 || o->max_iter_lm < 0)
    return SHAPE_EINVAL;
  if (!(o->k_gain > 0.0) || !(o->tol_x >= 0.0) || !(o->tol_g >= 0.0) || !(o->tol_lm >= 0.0))
    return SHAPE_EINVAL;
  if (!(o->gmax > 0.0 && o->gmax < 1.0) || !(o->lambda0 > 0.0) || !(o->chi2_rtol >= 0.0))
    return SHAPE_EINVAL;
  if (!(o->n0 >= 0.2 && o->n0 <= 10.0) || !(o->moffat_beta > 1.0)) return SHAPE_EINVAL;
  return SHAPE_OK;
}

KOpts kopts(const shape_opts* o) {
  KOpts k;
  k.max_iter_centroid = o->max_iter_centroid;
  k.max_iter_moments = o->max_iter_moments;
  k.max_iter_lm = o->max_iter_lm;
  k.free_mask = o->free_mask;
  k.k_gain = o->k_gain;
  k.tol_x = o->tol_x;
  k.tol_g = o->tol_g;
  k.gmax = o->gmax;
  k.tol_lm = o->tol_lm;
  k.lambda0 = o->lambda0;
  k.chi2_rtol = o->chi2_rtol;
  k.n0 = o->n0;
  k.moffat_beta = o->moffat_beta;
  k.linear_init = o->linear_init;
  return k;
}

int from_hip(hipError_t e) { return e == hipSuccess ? SHAPE_OK : SHAPE_EDEVICE; }

}  // namespace

extern "C" {

int shape_abi_version(void) { return SHAPE_ABI_VERSION; }

int shape_default_opts(shape_opts* o) {
  if (!o) return SHAPE_EINVAL;
  o->max_iter_centroid = 20;
  o->max_iter_moments = 20;
  o->max_iter_lm = 30;
  o->free_mask = 0xFFu;
  o->k_gain = 0.75;
  o->tol_x = 1e-4;
  o->tol_g = 1e-5;
  o->gmax = 0.95;
  o->tol_lm = 1e-5;
  o->lambda0 = 1e-3;
  o->chi2_rtol = 1e-6;
  o->n0 = 1.0;
  o->moffat_beta = 3.0;
  o->linear_init = 1;
  o->reserved = 0;
  return SHAPE_OK;
}

const char* shape_status_string(int code) {
  switch (code) {
    case SHAPE_OK: return "ok";
    case SHAPE_EINVAL: return "invalid argument";
    case SHAPE_EDEVICE: return "HIP device or launch error";
    case SHAPE_ENOMEM: return "workspace too small";
    case SHAPE_EUNSUPPORTED: return "unsupported option";
    default: return "unknown status";
  }
}

int shape_centroid(const shape_batch* b, const shape_opts* o, float* rec, int32_t* iters,
                   uint32_t* status, void* stream) {
  int rc = check_batch(b);
  if (rc == SHAPE_OK) rc = check_opts(o);
  if (rc != SHAPE_OK) return rc;
  if (b->n == 0) return SHAPE_OK;
  if (!rec || !iters || !status) return SHAPE_EINVAL;
  return from_hip(launch_centroid(*b, kopts(o), rec, iters, status, (hipStream_t)stream));
}

int shape_moments(const shape_batch* b, const shape_opts* o, const float* rec_in, float* rec_out,
                  int32_t* iters, uint32_t* status, void* stream) {
  int rc = check_batch(b);
  if (rc == SHAPE_OK) rc = check_opts(o);
  if (rc != SHAPE_OK) return rc;
  if (b->n == 0) return SHAPE_OK;
  if (!rec_in || !rec_out || !iters || !status) return SHAPE_EINVAL;
  return from_hip(
      launch_moments(*b, kopts(o), rec_in, rec_out, iters, status, (hipStream_t)stream));
}

int shape_fit_sersic(const shape_batch* b, const shape_opts* o, const float* p_init,
                     const float* rec, float* p_out, float* chi2, float* perr, int32_t* iters,
                     uint32_t* status, int32_t* sweeps, void* stream) {
  int rc = check_batch(b);
  if (rc == SHAPE_OK) rc = check_opts(o);
  if (rc != SHAPE_OK) return rc;
  if (o->free_mask != 0xFFu && o->free_mask != 0xF0u) return SHAPE_EUNSUPPORTED;
  if (!o->linear_init) return SHAPE_EUNSUPPORTED;
  if (b->n == 0) return SHAPE_OK;
  if ((!p_init && !rec) || !p_out || !chi2 || !iters || !status) return SHAPE_EINVAL;
  return from_hip(launch_fit(*b, kopts(o), p_init, rec, p_out, chi2, perr, iters, status,
                             sweeps, (hipStream_t)stream));
}

}  // extern "C"
