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
  if (!(o->gmax > 0.0 && o->gmax < 1.0) || !(o->lambda0 > 0.0) || !(o->chi2_rtol >= 0.0) ||
      !(o->tol_sigma >= 0.0))
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
  k.tol_sigma = o->tol_sigma;
  k.lambda0 = o->lambda0;
  k.chi2_rtol = o->chi2_rtol;
  k.n0 = o->n0;
  k.moffat_beta = o->moffat_beta;
  k.linear_init = o->linear_init;
  return k;
}

int from_hip(hipError_t e) { return e == hipSuccess ? SHAPE_OK : SHAPE_EDEVICE; }

int check_queue(const shape_batch* b, const shape_opts* o, const shape_queue_cfg* c,
                const void* ws, size_t ws_bytes) {
  int rc = check_batch(b);
  if (rc == SHAPE_OK) rc = check_opts(o);
  if (rc != SHAPE_OK) return rc;
  if (!c || (c->team != 1 && c->team != 2 && c->team != 4) || c->grid < 0) return SHAPE_EINVAL;
  if (c->chunk < 0 || c->chunk > 64) return SHAPE_EINVAL;
  if (c->team > 1 && (c->team_min_side < kMinSide || c->team_min_side > kMaxSide))
    return SHAPE_EINVAL;
  if (b->n > 0x7fffffffll) return SHAPE_EINVAL;
  if (o->free_mask != 0xFFu && o->free_mask != 0xF0u) return SHAPE_EUNSUPPORTED;
  if (o->free_mask == 0xF0u && c->team != 1) return SHAPE_EUNSUPPORTED;
  if (!o->linear_init) return SHAPE_EUNSUPPORTED;
  if (b->n == 0) return SHAPE_OK;
  if (!ws) return SHAPE_EINVAL;
  if (ws_bytes < queue_workspace_bytes(b->n)) return SHAPE_ENOMEM;
  return SHAPE_OK;
}

QCfg qcfg(const shape_queue_cfg* c) {
  QCfg q;
  q.team = c->team;
  q.team_min_side = c->team_min_side;
  q.grid = c->grid;
  q.chunk = c->chunk;
  return q;
}

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
  o->tol_sigma = 1e-4;
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
  // the unprofiled form exists for the 4-parameter Sersic fit only
  if (!o->linear_init && (o->free_mask != 0xF0u || b->model)) return SHAPE_EUNSUPPORTED;
  if (b->n == 0) return SHAPE_OK;
  if ((!p_init && !rec) || !p_out || !chi2 || !iters || !status) return SHAPE_EINVAL;
  return from_hip(launch_fit(*b, kopts(o), p_init, rec, p_out, chi2, perr, iters, status,
                             sweeps, (hipStream_t)stream));
}

int shape_chi2_fwd(const shape_batch* b, const float* params, float* chi2, void* stream) {
  int rc = check_batch(b);
  if (rc != SHAPE_OK) return rc;
  if (b->n == 0) return SHAPE_OK;
  if (!params || !chi2) return SHAPE_EINVAL;
  return from_hip(launch_chi2(*b, params, nullptr, chi2, nullptr, nullptr, nullptr, false,
                              (hipStream_t)stream));
}

int shape_chi2_bwd(const shape_batch* b, const float* params, const float* grad_chi2,
                   float* chi2, float* grad_p, float* jtj, float* jtr, void* stream) {
  int rc = check_batch(b);
  if (rc != SHAPE_OK) return rc;
  if (b->n == 0) return SHAPE_OK;
  if (!params || !grad_p) return SHAPE_EINVAL;
  return from_hip(
      launch_chi2(*b, params, grad_chi2, chi2, grad_p, jtj, jtr, true, (hipStream_t)stream));
}

int shape_chi2_grad_scale(const float* grad_unit, const float* grad_chi2, int64_t n,
                          float* grad_p, void* stream) {
  if (n < 0) return SHAPE_EINVAL;
  if (n == 0) return SHAPE_OK;
  if (!grad_unit || !grad_p) return SHAPE_EINVAL;
  return from_hip(launch_grad_scale(grad_unit, grad_chi2, n, grad_p, (hipStream_t)stream));
}

int shape_star_moments(const shape_batch* b, int32_t profile, const float* rec, double tol,
                       int32_t max_iter, float* out, int32_t* iters, uint32_t* status,
                       void* stream) {
  int rc = check_batch(b);
  if (rc != SHAPE_OK) return rc;
  if ((profile != 0 && profile != 1) || !(tol >= 0.0) || max_iter < 0) return SHAPE_EINVAL;
  if (b->n == 0) return SHAPE_OK;
  if (!rec || !out || !iters || !status) return SHAPE_EINVAL;
  return from_hip(
      launch_stars(*b, profile, rec, tol, max_iter, 3.0, out, iters, status, (hipStream_t)stream));
}

int shape_star_moments_beta(const shape_batch* b, double beta, const float* rec, double tol,
                            int32_t max_iter, float* out, int32_t* iters, uint32_t* status,
                            void* stream) {
  int rc = check_batch(b);
  if (rc != SHAPE_OK) return rc;
  if (!(beta > 1.0 && beta <= 1e6) || !(tol >= 0.0) || max_iter < 0) return SHAPE_EINVAL;
  if (b->n == 0) return SHAPE_OK;
  if (!rec || !out || !iters || !status) return SHAPE_EINVAL;
  return from_hip(
      launch_stars(*b, 2, rec, tol, max_iter, beta, out, iters, status, (hipStream_t)stream));
}

static int check_frames(const shape_frames* f) {
  if (!f || f->n < 0 || f->height < 4 || f->height > 4096 || f->width < 4 || f->width > 4096)
    return SHAPE_EINVAL;
  if (f->dtype != SHAPE_F32 && f->dtype != SHAPE_F16_SCALED) return SHAPE_EINVAL;
  if (f->n > 0 && (!f->pixels || (f->dtype == SHAPE_F16_SCALED && !f->scale))) return SHAPE_EINVAL;
  return SHAPE_OK;
}

int shape_frame_detect(const shape_frames* f, int32_t max_side, float* info, int32_t* peak,
                       int32_t* box, uint32_t* status, void* stream) {
  int rc = check_frames(f);
  if (rc != SHAPE_OK) return rc;
  if (max_side < 4 || max_side > 128) return SHAPE_EINVAL;
  if (f->n == 0) return SHAPE_OK;
  if (!info || !peak || !box || !status) return SHAPE_EINVAL;
  return from_hip(launch_frame_detect(*f, max_side, info, peak, box, status, (hipStream_t)stream));
}

int shape_frame_offsets(const int32_t* box, int64_t n, int64_t* offset, int64_t* total,
                        void* stream) {
  if (n < 0 || !total || (n > 0 && (!box || !offset))) return SHAPE_EINVAL;
  return from_hip(launch_frame_offsets(box, n, offset, total, (hipStream_t)stream));
}

int shape_frame_cut(const shape_frames* f, const int32_t* box, const int64_t* offset,
                    float* stamps, int64_t capacity, int32_t* sides, void* stream) {
  int rc = check_frames(f);
  if (rc != SHAPE_OK) return rc;
  if (capacity < 0) return SHAPE_EINVAL;
  if (f->n == 0) return SHAPE_OK;
  if (!box || !offset || !stamps) return SHAPE_EINVAL;
  return from_hip(
      launch_frame_cut(*f, box, offset, stamps, capacity, sides, (hipStream_t)stream));
}

int shape_queue_default_cfg(shape_queue_cfg* c) {
  if (!c) return SHAPE_EINVAL;
  c->team = 1;
  c->team_min_side = 96;
  c->grid = 0;
  c->chunk = 0;
  return SHAPE_OK;
}

int shape_queue_workspace_bytes(int64_t n, size_t* bytes) {
  if (n < 0 || !bytes) return SHAPE_EINVAL;
  *bytes = queue_workspace_bytes(n);
  return SHAPE_OK;
}

int shape_queue_start(const shape_batch* b, const shape_opts* o, const shape_queue_cfg* c,
                      const float* p_init, const float* rec, void* ws, size_t ws_bytes,
                      void* stream) {
  int rc = check_queue(b, o, c, ws, ws_bytes);
  if (rc != SHAPE_OK || b->n == 0) return rc;
  if (!p_init && !rec) return SHAPE_EINVAL;
  return from_hip(launch_queue_start(*b, kopts(o), ws, p_init, rec, qcfg(c), (hipStream_t)stream));
}

int shape_queue_step(const shape_batch* b, const shape_opts* o, const shape_queue_cfg* c, void* ws,
                     size_t ws_bytes, void* stream) {
  int rc = check_queue(b, o, c, ws, ws_bytes);
  if (rc != SHAPE_OK || b->n == 0) return rc;
  return from_hip(launch_queue_step(*b, kopts(o), ws, qcfg(c), (hipStream_t)stream));
}

int shape_queue_drain(const shape_batch* b, const shape_opts* o, const shape_queue_cfg* c, void* ws,
                      size_t ws_bytes, void* stream) {
  int rc = check_queue(b, o, c, ws, ws_bytes);
  if (rc != SHAPE_OK || b->n == 0) return rc;
  return from_hip(launch_queue_drain(*b, kopts(o), ws, qcfg(c), (hipStream_t)stream));
}

int shape_queue_finish(const shape_batch* b, const shape_opts* o, void* ws, size_t ws_bytes,
                       float* p_out, float* chi2, float* perr, int32_t* iters, uint32_t* status,
                       int32_t* sweeps, void* stream) {
  shape_queue_cfg c;
  shape_queue_default_cfg(&c);
  int rc = check_queue(b, o, &c, ws, ws_bytes);
  if (rc != SHAPE_OK || b->n == 0) return rc;
  if (!p_out || !chi2 || !iters || !status) return SHAPE_EINVAL;
  return from_hip(launch_queue_finish(*b, kopts(o), ws, p_out, chi2, perr, iters, status, sweeps,
                                      (hipStream_t)stream));
}

int shape_fit_queue_static(const shape_batch* b, const shape_opts* o, const shape_queue_cfg* c,
                           const float* p_init, const float* rec, float* p_out, float* chi2,
                           float* perr, int32_t* iters, uint32_t* status, int32_t* sweeps,
                           void* stream) {
  if (b && b->n > SHAPE_STATIC_MAX_STAMPS) return SHAPE_ENOMEM;
  // the workspace checks of check_queue are met by the static array
  int rc = check_queue(b, o, c, reinterpret_cast<void*>(1), static_queue_scratch_bytes());
  if (rc != SHAPE_OK || b->n == 0) return rc;
  if ((!p_init && !rec) || !p_out || !chi2 || !iters || !status) return SHAPE_EINVAL;
  return from_hip(launch_fit_queue_static(*b, kopts(o), p_init, rec, qcfg(c), p_out, chi2, perr,
                                          iters, status, sweeps, (hipStream_t)stream));
}

struct shape_queue_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

int shape_queue_graph_create(const shape_batch* b, const shape_opts* o, const shape_queue_cfg* c,
                             void* ws, size_t ws_bytes, shape_queue_graph** out) {
  if (!out) return SHAPE_EINVAL;
  *out = nullptr;
  int rc = check_queue(b, o, c, ws, ws_bytes);
  if (rc != SHAPE_OK) return rc;
  if (b->n == 0) return SHAPE_EINVAL;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return SHAPE_EDEVICE;
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t le = launch_queue_step(*b, kopts(o), ws, qcfg(c), s);
    e = hipStreamEndCapture(s, &g);
    if (le != hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipStreamDestroy(s);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return SHAPE_EDEVICE;
  }
  *out = new shape_queue_graph{g, x};
  return SHAPE_OK;
}

int shape_queue_graph_launch(shape_queue_graph* g, void* stream) {
  if (!g) return SHAPE_EINVAL;
  return from_hip(hipGraphLaunch(g->exec, (hipStream_t)stream));
}

int shape_queue_graph_destroy(shape_queue_graph* g) {
  if (!g) return SHAPE_EINVAL;
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  delete g;
  return SHAPE_OK;
}

}  // extern "C"
