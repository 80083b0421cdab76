// Adaptive interpolation interval (Sec. 3.3): host-side policy that decides,
// frame by frame, between a real render and a reprojected frame. The
// interval (frames per real render, at most four) follows the measured frame
// costs so the mean frame time meets a target with as little interpolation
// as possible; when even the longest interval cannot meet it, rendering
// falls back to every frame real.
#include <cmath>

#include "internal.h"

namespace {

int choose_interval(const starnt_interval& s) {
  if (s.real_ms < 0.0 || s.real_ms <= s.target_ms) return 1;
  if (s.max_interval < 2) return 1;
  if (s.interp_ms < 0.0) return 2;  // probe: measure one interpolated frame
  for (int k = 2; k <= s.max_interval; ++k)
    if ((s.real_ms + (k - 1) * s.interp_ms) / k <= s.target_ms) return k;
  return 1;  // the target is out of reach: standard rendering
}

}  // namespace

extern "C" {

int starnt_interval_init(starnt_interval* s, double target_ms, int32_t max_interval, double smoothing) {
  if (!s) return starnt::fail(STARNT_EINVAL, "starnt_interval_init: NULL state");
  if (!(target_ms > 0.0) || !std::isfinite(target_ms))
    return starnt::fail(STARNT_EINVAL, "starnt_interval_init: target_ms must be positive");
  if (max_interval < 1 || max_interval > 4)
    return starnt::fail(STARNT_EINVAL, "starnt_interval_init: max_interval must be in 1..4");
  if (!(smoothing > 0.0 && smoothing <= 1.0))
    return starnt::fail(STARNT_EINVAL, "starnt_interval_init: smoothing must be in (0, 1]");
  s->target_ms = target_ms;
  s->smoothing = smoothing;
  s->real_ms = -1.0;
  s->interp_ms = -1.0;
  s->max_interval = max_interval;
  s->interval = 1;
  s->pos = 0;
  s->pad = 0;
  return STARNT_OK;
}

int starnt_interval_next(starnt_interval* s) {
  if (!s) return -1;
  if (s->pos == 0) s->interval = choose_interval(*s);
  const int real = s->pos == 0 ? 1 : 0;
  s->pos = (s->pos + 1) % s->interval;
  return real;
}

int starnt_interval_report(starnt_interval* s, int32_t was_real, double ms) {
  if (!s) return starnt::fail(STARNT_EINVAL, "starnt_interval_report: NULL state");
  if (!(ms >= 0.0) || !std::isfinite(ms))
    return starnt::fail(STARNT_EINVAL, "starnt_interval_report: time must be finite and >= 0");
  double& m = was_real ? s->real_ms : s->interp_ms;
  m = m < 0.0 ? ms : m + s->smoothing * (ms - m);
  return STARNT_OK;
}

}  // extern "C"
