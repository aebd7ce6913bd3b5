// Step-size control of the adaptive reaction stage (paper section 3.3.1: the
// embedded ROS2 solution chooses the next step; section 4: adaptive steps
// capped at a maximum).  One step size serves every vertex of the run, as the
// tissue shares one step in the partitioned strategy.  The controller lives on
// the device so that attempts queue back to back on the stream: each attempt
// is one step kernel (which raises the error slots to its largest lane
// errors) followed by adapt_control_kernel, which folds and clears the slots
// and then
//   * accepts the attempt iff err <= tol (a non-finite err rejects it),
//     advancing t (exactly to the breakpoint when the step was cut to one) and
//     flipping the buffer holding the state;
//   * sets the proposed step to tau * min(2, max(0.2, 0.9 (tol/err)^(1/2)))
//     (err == 0: factor 2; non-finite: 0.2), capped at dt_max;
//   * plans the next attempt: the step is cut to reach the next breakpoint
//     (stimulus switching times, t_end) when it would reach or cross it; the
//     run is done at t_end, failed when the step falls below dt_min or the
//     attempts run out.
#include "kernel_ops.h"

namespace ionic {

namespace {

constexpr double kSafety = 0.9;
constexpr double kQMin = 0.2;
constexpr double kQMax = 2.0;

__device__ void plan_next(AdaptCtl* c) {
  if (c->t >= c->t_end) {
    c->done = 1;
    return;
  }
  if (c->attempts >= c->max_attempts) {
    c->done = 1;
    c->failed = 1;
    return;
  }
  double b = c->t_end;
  if (c->t < c->t_on && c->t_on < b) b = c->t_on;
  if (c->t < c->t_off && c->t_off < b) b = c->t_off;
  const int hit = c->dt_try >= b - c->t;
  const double tau = hit ? b - c->t : c->dt_try;
  if (tau < c->dt_min) {
    c->done = 1;
    c->failed = 1;
    return;
  }
  c->b = b;
  c->hit = hit;
  c->tau = tau;
}

__global__ void adapt_init_kernel(AdaptCtl* c, ErrSlot* err, double t0, double t_end, double dt_init,
                                  double dt_max, double tol, double dt_min, double t_on,
                                  double t_off, long long max_attempts) {
  if (threadIdx.x < kSlots) err[threadIdx.x].bits = 0ull;
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  c->t = t0;
  c->t_end = t_end;
  c->dt_max = dt_max;
  c->dt_try = dt_init < dt_max ? dt_init : dt_max;
  c->tol = tol;
  c->dt_min = dt_min;
  c->t_on = t_on;
  c->t_off = t_off;
  c->err_last = 0.0;
  c->accepted = 0;
  c->rejected = 0;
  c->attempts = 0;
  c->max_attempts = max_attempts;
  c->cur = 0;
  c->done = 0;
  c->failed = 0;
  c->hit = 0;
  c->tau = 0.0;
  c->b = t_end;
  plan_next(c);
}

// one wavefront: lane l folds and clears slot l, lane 0 decides
__global__ void adapt_control_kernel(AdaptCtl* c, ErrSlot* slots, double* history,
                                     long long history_len) {
  static_assert(kSlots == 64, "one slot per lane of the control wavefront");
  if (c->done) return;
  const unsigned long long mine = slots[threadIdx.x].bits;
  slots[threadIdx.x].bits = 0ull;
  const unsigned long long bits = wave_max_u64(mine);
  if (threadIdx.x != 0) return;
  const double err = __longlong_as_double((long long)bits);
  const bool finite = err <= 1.0e308;
  const bool ok = finite && err <= c->tol;
  const long long a = c->attempts;
  if (history && a < history_len) {
    history[4 * a + 0] = c->t;
    history[4 * a + 1] = c->tau;
    history[4 * a + 2] = err;
    history[4 * a + 3] = ok ? 1.0 : 0.0;
  }
  c->attempts = a + 1;
  c->err_last = err;
  double q;
  if (!finite)
    q = kQMin;
  else if (err == 0.0)
    q = kQMax;
  else {
    q = kSafety * ::sqrt(c->tol / err);
    q = q < kQMin ? kQMin : (q > kQMax ? kQMax : q);
  }
  if (ok) {
    c->t = c->hit ? c->b : c->t + c->tau;
    c->accepted += 1;
    c->cur ^= 1;
  } else {
    c->rejected += 1;
  }
  const double next = c->tau * q;
  c->dt_try = next < c->dt_max ? next : c->dt_max;
  plan_next(c);
}

}  // namespace

hipError_t adapt_init(AdaptCtl* c, ErrSlot* err, double t0, double t_end, double dt_init,
                      double dt_max, double tol, double dt_min, double t_on, double t_off,
                      long long max_attempts, hipStream_t st) {
  hipLaunchKernelGGL(adapt_init_kernel, dim3(1), dim3(kSlots), 0, st, c, err, t0, t_end, dt_init,
                     dt_max, tol, dt_min, t_on, t_off, max_attempts);
  return hipGetLastError();
}

hipError_t adapt_control(AdaptCtl* c, ErrSlot* err, double* history, long long history_len,
                         hipStream_t st) {
  hipLaunchKernelGGL(adapt_control_kernel, dim3(1), dim3(kSlots), 0, st, c, err, history,
                     history_len);
  return hipGetLastError();
}

}  // namespace ionic
