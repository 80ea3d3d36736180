// Adaptive keyframe selection (CaRtGS Sec. III-C-2, Eqs. (5)-(8)), host side.
// Keyframes enter with r0 remaining optimisations; each mapping iteration
// draws keyframes uniformly among those with r > 0 (the caller supplies the
// uniform draws), decrements their counts and later reports their losses;
// when no keyframe is left, the counts are reset to 2 for the d_k largest
// losses and 1 for the rest, d_k = max(1, floor(k / d)), ties to the lower
// keyframe index.  A new keyframe's loss is +inf until reported.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/gs.h"

namespace {
thread_local char g_msg[256];
gs_status bad(const char* m) {
  std::strncpy(g_msg, m, sizeof g_msg - 1);
  return GS_ERR_INVALID_ARG;
}
}  // namespace

extern "C" {

const char* gs_sched_last_error(void) { return g_msg; }

gs_status gs_sched_init(gs_scheduler* s, int32_t* r, double* l, int32_t capacity, int32_t r0,
                        int32_t d) {
  if (!s || !r || !l) return bad("null argument");
  if (capacity < 1 || r0 < 1 || d < 1) return bad("capacity, r0 and d must be >= 1");
  s->r = r;
  s->l = l;
  s->capacity = capacity;
  s->count = 0;
  s->r0 = r0;
  s->d = d;
  s->refills = 0;
  return GS_OK;
}

gs_status gs_sched_add_keyframe(gs_scheduler* s, int32_t* out_id) {
  if (!s || !s->r) return bad("scheduler not initialised");
  if (s->count >= s->capacity) return bad("keyframe capacity reached");
  const int32_t i = s->count++;
  s->r[i] = s->r0;
  s->l[i] = INFINITY;
  if (out_id) *out_id = i;
  return GS_OK;
}

static void refill(gs_scheduler* s) {
  const int32_t k = s->count;
  const int32_t dk = std::max(1, k / s->d);
  std::vector<int32_t> idx(k);
  for (int32_t i = 0; i < k; ++i) idx[i] = i;
  const double* l = s->l;
  std::partial_sort(idx.begin(), idx.begin() + std::min(dk, k), idx.end(),
                    [l](int32_t a, int32_t b) { return l[a] > l[b] || (l[a] == l[b] && a < b); });
  for (int32_t i = 0; i < k; ++i) s->r[i] = 1;
  for (int32_t j = 0; j < std::min(dk, k); ++j) s->r[idx[j]] = 2;
  s->refills += 1;
}

gs_status gs_sched_select(gs_scheduler* s, int32_t batch, const double* uniforms,
                          int32_t* out_ids, int32_t* out_count) {
  if (!s || !s->r) return bad("scheduler not initialised");
  if (batch < 0 || (batch > 0 && (!uniforms || !out_ids)) || !out_count) return bad("bad batch arguments");
  *out_count = 0;
  if (s->count == 0 || batch == 0) return GS_OK;
  bool any = false;
  for (int32_t i = 0; i < s->count; ++i) any = any || s->r[i] > 0;
  if (!any) refill(s);
  std::vector<int32_t> elig;
  for (int32_t i = 0; i < s->count; ++i)
    if (s->r[i] > 0) elig.push_back(i);
  int32_t n = 0;
  for (int32_t b = 0; b < batch && !elig.empty(); ++b) {
    const double u = uniforms[b];
    if (!(u >= 0.0 && u < 1.0)) return bad("uniform draws must lie in [0, 1)");
    size_t j = (size_t)std::floor(u * (double)elig.size());
    if (j >= elig.size()) j = elig.size() - 1;
    out_ids[n++] = elig[j];
    elig.erase(elig.begin() + (long)j);
  }
  for (int32_t k = 0; k < n; ++k) s->r[out_ids[k]] -= 1;
  *out_count = n;
  return GS_OK;
}

gs_status gs_sched_report(gs_scheduler* s, int32_t id, double loss) {
  if (!s || !s->r) return bad("scheduler not initialised");
  if (id < 0 || id >= s->count) return bad("keyframe id out of range");
  s->l[id] = loss;
  return GS_OK;
}

}  // extern "C"
