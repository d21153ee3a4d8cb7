// Reverse-mode differentiation of a run of the coupled step (C ABI of the
// tape; declarations and contracts in include/lbf.h).
//
// The forward run stores the state every `segment` steps (sqrt(N) by
// default).  The backward sweep walks the segments from last to first:
// recompute the segment from its checkpoint with the step kernel (which also
// stores phi, f_s and rho of every state for the reverse stencils), then
// run the two adjoint kernels per step in reverse order.  The recomputation
// of segment k - 1 does not depend on the adjoint, so it runs on a second
// stream into the other of two segment buffers while segment k is reversed;
// events order each buffer's reuse.  Gradients are accumulated in FP64 on
// the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>

#include "lbf.h"
#include "lbf_adjoint.hpp"
#include "lbf_sim.hpp"

using namespace lbf;
using namespace lbfi;

namespace {

constexpr int kStatePlanes = NDIST + NLAG;   // one stored state: D then L

}  // namespace

struct lbf_tape {
  lbf_sim* sim;
  int nsteps, seg, nck;
  size_t P;               // plane stride (floats)
  char* mem;
  size_t bytes;
  float* ck;              // nck states
  float* segs[2];         // seg states each (recomputed segments, alternating)
  float* mom[2];          // seg x 3 planes each
  float* adjD[2];         // NADJ_D planes per time-level parity
  float* adjL[2];         // NADJ_L planes
  float* st;              // NST planes
  float* jac;             // NJAC planes
  float* seeds;           // 3 planes (staging of host seeds)
  double* gcth;           // nx * ny
  double* gwall;          // 4 * wstride
  hipStream_t rstream;    // recomputation stream (default priority)
  hipEvent_t ev_start, ev_rec[2], ev_used[2];
  bool recorded;          // forward run done, sim at its final state
  bool with_init;         // the run started from lbf_init_fields
  long long end_step;     // sim step count after the recorded run
};

namespace {

constexpr int kTapeParts = 14;

size_t tape_layout(int nx, int ny, long long plane, int nsteps, int seg,
                   size_t offs[kTapeParts]) {
  const size_t P = (size_t)plane * sizeof(float);
  const int nck = (nsteps + seg - 1) / seg;
  const size_t wstride = round_up((size_t)std::max(nx, ny), 64);
  size_t off = 0;
  int q = 0;
  auto take = [&](size_t b) {
    offs[q++] = off;
    off = round_up(off + b, kAlign);
  };
  take((size_t)std::max(nck, 1) * kStatePlanes * P);   // 0 checkpoints
  take((size_t)seg * kStatePlanes * P);                // 1, 2 segment states
  take((size_t)seg * kStatePlanes * P);
  take((size_t)seg * 3 * P);                           // 3, 4 segment moments
  take((size_t)seg * 3 * P);
  take(NADJ_D * P);                                    // 5, 6
  take(NADJ_D * P);
  take(NADJ_L * P);                                    // 7, 8
  take(NADJ_L * P);
  take(NST * P);                                       // 9
  take(NJAC * P);                                      // 10
  take(3 * P);                                         // 11 seeds
  take((size_t)nx * ny * sizeof(double));              // 12 gcth
  take(4 * wstride * sizeof(double));                  // 13 gwall
  return off;
}

int default_segment(int nsteps) {
  return std::max(1, (int)std::ceil(std::sqrt((double)std::max(nsteps, 1))));
}

// state slot `idx` of the checkpoints (kind 0) or of segment buffer kind - 1
float* state_ptr(lbf_tape* t, int kind, int idx) {
  float* base = kind == 0 ? t->ck : t->segs[kind - 1];
  return base + (size_t)idx * kStatePlanes * t->P;
}

BufArgs state_args(lbf_tape* t, const float* st) {
  lbf_sim* s = t->sim;
  BufArgs B{};
  B.din = st;
  B.lin = st + NDIST * t->P;
  B.stat = fptr(s, s->L.stat);
  B.wallT = fptr(s, s->L.wall);
  B.wstride = s->L.wstride;
  B.dout = nullptr;
  B.lout = nullptr;
  B.fields = nullptr;
  B.red = nullptr;
  return B;
}

dim3 adj_grid(const lbf_sim* s) { return dim3((s->G.nx + 255) / 256, s->G.ny, 1); }

int copy_state_out(lbf_tape* t, float* dst) {
  lbf_sim* s = t->sim;
  const size_t pb = t->P * sizeof(float);
  HIP_TRY(hipMemcpyAsync(dst, s->ws + s->L.dist[s->cur], NDIST * pb, hipMemcpyDeviceToDevice,
                         s->stream));
  HIP_TRY(hipMemcpyAsync(dst + NDIST * t->P, s->ws + s->L.lag[s->cur], NLAG * pb,
                         hipMemcpyDeviceToDevice, s->stream));
  return LBF_OK;
}

// Step state `in` to `out` with the step kernel, storing phi, f_s, rho of
// `in` in `mom`, on stream `st`.
int recompute_step(lbf_tape* t, const float* in, float* out, float* mom, hipStream_t st) {
  lbf_sim* s = t->sim;
  BufArgs B = state_args(t, in);
  B.dout = out;
  B.lout = out + NDIST * t->P;
  B.fields = mom;
  return launch_step_args(s, MODE_STEP_MOM, false, B, st);
}

// Recompute segment `sgi` (states c + 1 .. c + L - 1 and the moments of
// c .. c + L - 1) into buffer sgi & 1 on the recomputation stream, after the
// buffer's previous reader has finished.
int recompute_segment(lbf_tape* t, int sgi, bool buffer_used) {
  const int b = sgi & 1;
  const int c = sgi * t->seg;
  const int L = std::min(t->seg, t->nsteps - c);
  if (buffer_used) HIP_TRY(hipStreamWaitEvent(t->rstream, t->ev_used[b], 0));
  for (int j = 0; j < L; ++j) {
    const float* in = j == 0 ? state_ptr(t, 0, sgi) : state_ptr(t, 1 + b, j - 1);
    int rc = recompute_step(t, in, state_ptr(t, 1 + b, j), t->mom[b] + (size_t)j * 3 * t->P,
                            t->rstream);
    if (rc) return rc;
  }
  HIP_TRY(hipEventRecord(t->ev_rec[b], t->rstream));
  return LBF_OK;
}

}  // namespace

extern "C" {

size_t lbf_tape_bytes(int32_t nx, int32_t ny, int32_t plane_pad, int32_t nsteps,
                      int32_t segment) {
  if (nx < 1 || ny < 1 || nsteps < 0 || plane_pad < 0 || plane_pad > kMaxPlanePad ||
      plane_pad % 64)
    return 0;
  const int seg = segment > 0 ? segment : default_segment(nsteps);
  size_t offs[kTapeParts];
  return tape_layout(nx, ny, plane_stride(nx, ny, plane_pad, 0), nsteps, seg, offs);
}

int lbf_tape_create(lbf_sim* sim, int32_t nsteps, int32_t segment, lbf_tape** out) {
  if (!out) return fail(LBF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!sim) return fail(LBF_EINVAL, "sim is NULL");
  if (sim->prm.mrt) return fail(LBF_EINVAL, "the adjoint supports the BGK flow collision only");
  if (sim->prm.grav[0] != 0.0 || sim->prm.grav[1] != 0.0 || sim->prm.u_solid[0] != 0.0 ||
      sim->prm.u_solid[1] != 0.0)
    return fail(LBF_EINVAL, "the adjoint supports grav = u_solid = 0 only");
  if (sim->ph.subfix == 2)
    return fail(LBF_EINVAL, "the adjoint supports the phi0 >= 1/2 held region only, not a "
                            "per-node isothermal region");
  if (sim->ph.phi_src_flow)
    return fail(LBF_EINVAL, "the adjoint supports phi_src_mdot = 1 only (the phase-field "
                            "source from the mass source)");
  if (sim->prm.row_block != 0)
    return fail(LBF_EINVAL, "the adjoint supports row_block = 0 (the plane-major layout) only");
  if (nsteps < 0) return fail(LBF_EINVAL, "nsteps %d", nsteps);
  if (segment < 0) return fail(LBF_EINVAL, "segment %d", segment);
  lbf_tape* t = new (std::nothrow) lbf_tape();
  if (!t) return fail(LBF_ENOMEM, "host allocation failed");
  t->sim = sim;
  t->nsteps = nsteps;
  t->seg = segment > 0 ? std::min<int>(segment, std::max(nsteps, 1)) : default_segment(nsteps);
  t->nck = (nsteps + t->seg - 1) / t->seg;
  t->P = (size_t)sim->G.P;
  size_t offs[kTapeParts];
  t->bytes = tape_layout(sim->G.nx, sim->G.ny, sim->G.P, nsteps, t->seg, offs);
  if (hipMalloc((void**)&t->mem, t->bytes) != hipSuccess) {
    const size_t b = t->bytes;
    delete t;
    return fail(LBF_ENOMEM, "hipMalloc of %zu tape bytes failed", b);
  }
  auto F = [&](int q) { return reinterpret_cast<float*>(t->mem + offs[q]); };
  t->ck = F(0);
  t->segs[0] = F(1);
  t->segs[1] = F(2);
  t->mom[0] = F(3);
  t->mom[1] = F(4);
  t->adjD[0] = F(5);
  t->adjD[1] = F(6);
  t->adjL[0] = F(7);
  t->adjL[1] = F(8);
  t->st = F(9);
  t->jac = F(10);
  t->seeds = F(11);
  t->gcth = reinterpret_cast<double*>(t->mem + offs[12]);
  t->gwall = reinterpret_cast<double*>(t->mem + offs[13]);
  bool ok = hipStreamCreateWithFlags(&t->rstream, hipStreamNonBlocking) == hipSuccess;
  for (hipEvent_t* e : {&t->ev_start, &t->ev_rec[0], &t->ev_rec[1], &t->ev_used[0], &t->ev_used[1]})
    ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    lbf_tape_destroy(t);
    return fail(LBF_EHIP, "stream / event creation failed");
  }
  *out = t;
  return LBF_OK;
}

int lbf_tape_segment(const lbf_tape* t) { return t ? t->seg : 0; }

int lbf_tape_forward(lbf_tape* t) {
  if (!t) return fail(LBF_EINVAL, "tape is NULL");
  lbf_sim* s = t->sim;
  if (!s->have_init) return fail(LBF_ESTATE, "the simulation is not initialised");
  if (s->ph.subfix == 2)
    return fail(LBF_EINVAL, "the adjoint supports the phi0 >= 1/2 held region only, not a "
                            "per-node isothermal region");
  t->with_init = s->from_fields && s->step == 0;
  for (int c = 0; c < t->nsteps; c += t->seg) {
    int rc = copy_state_out(t, state_ptr(t, 0, c / t->seg));
    if (rc) return rc;
    rc = lbf_step(s, std::min(t->seg, t->nsteps - c));
    if (rc) return rc;
  }
  t->recorded = true;
  t->end_step = s->step;
  return LBF_OK;
}

int lbf_tape_backward(lbf_tape* t, const float* seed_phi, const float* seed_T,
                      const float* seed_fs, int32_t seeds_on_device, double* grad_cos_theta,
                      double* grad_wall_T, int32_t grads_on_device) {
  if (!t) return fail(LBF_EINVAL, "tape is NULL");
  if (!grad_cos_theta || !grad_wall_T) return fail(LBF_EINVAL, "NULL gradient output");
  lbf_sim* s = t->sim;
  if (!t->recorded) return fail(LBF_ESTATE, "lbf_tape_forward must precede lbf_tape_backward");
  if (s->step != t->end_step)
    return fail(LBF_ESTATE, "the simulation moved since the recorded run (step %lld, expected %lld)",
                s->step, t->end_step);
  const int nx = s->G.nx, ny = s->G.ny;
  const size_t n = (size_t)nx * ny;
  const size_t P = t->P;
  hipStream_t st = s->stream;
  // seeds
  const float* sd[3] = {seed_phi, seed_T, seed_fs};
  if (!seeds_on_device) {
    for (int q = 0; q < 3; ++q) {
      if (!sd[q]) continue;
      HIP_TRY(hipMemcpyAsync(t->seeds + q * P, sd[q], n * sizeof(float), hipMemcpyHostToDevice,
                             st));
      sd[q] = t->seeds + q * P;
    }
    HIP_TRY(hipStreamSynchronize(st));
  }
  HIP_TRY(hipMemsetAsync(t->gcth, 0, n * sizeof(double), st));
  HIP_TRY(hipMemsetAsync(t->gwall, 0, 4 * (size_t)s->L.wstride * sizeof(double), st));
  const dim3 grid = adj_grid(s), block(256);
  const int N = t->nsteps;
  // seed at the final state (the simulation's current state)
  {
    AdjSeedArgs a{};
    a.G = s->G;
    a.ph = s->ph;
    a.F = state_args(t, fptr(s, s->L.dist[s->cur]));
    a.F.lin = fptr(s, s->L.lag[s->cur]);
    a.sphi = sd[0];
    a.sT = sd[1];
    a.sfs = sd[2];
    a.outD = t->adjD[N & 1];
    a.outL = t->adjL[N & 1];
    hipLaunchKernelGGL(k_adj_seed, grid, block, 0, st, a);
    HIP_TRY(hipGetLastError());
  }
  // both streams start after everything queued so far on the simulation's stream
  HIP_TRY(hipEventRecord(t->ev_start, st));
  HIP_TRY(hipStreamWaitEvent(t->rstream, t->ev_start, 0));
  if (t->nck > 0) {
    int rc = recompute_segment(t, t->nck - 1, false);
    if (rc) return rc;
  }
  for (int sgi = t->nck - 1; sgi >= 0; --sgi) {
    const int b = sgi & 1;
    const int c = sgi * t->seg;
    const int L = std::min(t->seg, N - c);
    // the next segment to reverse is recomputed while this one is reversed
    if (sgi > 0) {
      int rc = recompute_segment(t, sgi - 1, sgi + 1 < t->nck);
      if (rc) return rc;
    }
    HIP_TRY(hipStreamWaitEvent(st, t->ev_rec[b], 0));
    for (int j = L - 1; j >= 0; --j) {
      const int nstep = c + j;
      const float* stn = j == 0 ? state_ptr(t, 0, sgi) : state_ptr(t, 1 + b, j - 1);
      AdjStepArgs a{};
      a.G = s->G;
      a.ph = s->ph;
      a.F = state_args(t, stn);
      a.mom = t->mom[b] + (size_t)j * 3 * P;
      a.lamD = t->adjD[(nstep + 1) & 1];
      a.lamL = t->adjL[(nstep + 1) & 1];
      a.outD = t->adjD[nstep & 1];
      a.outL = t->adjL[nstep & 1];
      a.st = t->st;
      a.jac = t->jac;
      a.gcth = t->gcth;
      a.gwall = t->gwall;
      hipLaunchKernelGGL(k_adj_collide, grid, block, 0, st, a);
      HIP_TRY(hipGetLastError());
      AdjGatherArgs g{};
      g.G = s->G;
      g.st = t->st;
      g.jac = t->jac;
      g.outD = t->adjD[nstep & 1];
      g.outL = t->adjL[nstep & 1];
      hipLaunchKernelGGL(k_adj_gather, grid, block, 0, st, g);
      HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipEventRecord(t->ev_used[b], st));
  }
  if (t->with_init) {
    AdjInitArgs a{};
    a.G = s->G;
    a.ph = s->ph;
    // the initial state: checkpoint 0, or the current state of a run of 0 steps
    a.F = N > 0 ? state_args(t, state_ptr(t, 0, 0)) : state_args(t, fptr(s, s->L.dist[s->cur]));
    if (N == 0) a.F.lin = fptr(s, s->L.lag[s->cur]);
    a.lamD = t->adjD[0];
    a.gcth = t->gcth;
    hipLaunchKernelGGL(k_adj_init, grid, block, 0, st, a);
    HIP_TRY(hipGetLastError());
  }
  // outputs: cos(theta) per node; wall profiles bottom (nx), top (nx), left (ny), right (ny)
  const hipMemcpyKind kind = grads_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  HIP_TRY(hipMemcpyAsync(grad_cos_theta, t->gcth, n * sizeof(double), kind, st));
  const size_t ws = (size_t)s->L.wstride;
  HIP_TRY(hipMemcpyAsync(grad_wall_T, t->gwall, nx * sizeof(double), kind, st));
  HIP_TRY(hipMemcpyAsync(grad_wall_T + nx, t->gwall + ws, nx * sizeof(double), kind, st));
  HIP_TRY(hipMemcpyAsync(grad_wall_T + 2 * nx, t->gwall + 2 * ws, ny * sizeof(double), kind, st));
  HIP_TRY(hipMemcpyAsync(grad_wall_T + 2 * nx + ny, t->gwall + 3 * ws, ny * sizeof(double), kind,
                         st));
  HIP_TRY(hipStreamSynchronize(st));
  return LBF_OK;
}

void lbf_tape_destroy(lbf_tape* t) {
  if (!t) return;
  if (t->sim && t->sim->stream) (void)hipStreamSynchronize(t->sim->stream);
  else (void)hipDeviceSynchronize();
  if (t->rstream) {
    (void)hipStreamSynchronize(t->rstream);
    (void)hipStreamDestroy(t->rstream);
  }
  for (hipEvent_t e : {t->ev_start, t->ev_rec[0], t->ev_rec[1], t->ev_used[0], t->ev_used[1]})
    if (e) (void)hipEventDestroy(e);
  if (t->mem) (void)hipFree(t->mem);
  delete t;
}

}  // extern "C"
