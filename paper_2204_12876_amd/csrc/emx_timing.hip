// Optional per-kernel timing.
//
// While timing is on, every kernel the library launches directly is bracketed
// by two timing events recorded on the kernel's own stream.  emx_timing_end
// waits for them and reports, per kernel, the number of launches and the
// summed duration.  Launches into a stream that is being captured into a graph
// are not timed.  Timing is meant for one host thread driving the library.
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "emx_host.h"

namespace emx {

namespace {

struct Mark {
  const char* name;
  hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Mark> g_marks;      // recorded since emx_timing_begin
std::vector<hipEvent_t> g_free;  // reusable events

hipEvent_t take_event() {
  if (!g_free.empty()) {
    hipEvent_t e = g_free.back();
    g_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

TimedLaunch::TimedLaunch(const char* name, hipStream_t s) : stream_(s), idx_(-1) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  Mark m{name, take_event(), take_event()};
  if (!m.a || !m.b || hipEventRecord(m.a, s) != hipSuccess) {
    if (m.a) g_free.push_back(m.a);
    if (m.b) g_free.push_back(m.b);
    return;
  }
  idx_ = (long)g_marks.size();
  g_marks.push_back(m);
}

TimedLaunch::~TimedLaunch() {
  if (idx_ < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (idx_ < (long)g_marks.size()) (void)hipEventRecord(g_marks[idx_].b, stream_);
}

}  // namespace emx

using namespace emx;

extern "C" {

emx_status emx_timing_begin(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (const Mark& m : g_marks) {
    g_free.push_back(m.a);
    g_free.push_back(m.b);
  }
  g_marks.clear();
  g_on = true;
  return EMX_OK;
}

emx_status emx_timing_end(char* buf, size_t len) {
  if (!buf || len == 0) return fail(EMX_EINVAL, "buf is NULL");
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = false;
  // sum per kernel name, in order of first launch
  std::vector<const char*> names;
  std::vector<long> count;
  std::vector<double> total;
  for (const Mark& m : g_marks) {
    hipError_t e = hipEventSynchronize(m.b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, m.a, m.b);
    if (e != hipSuccess) return hip_fail(e, "timing_end");
    size_t k = 0;
    while (k < names.size() && strcmp(names[k], m.name) != 0) ++k;
    if (k == names.size()) {
      names.push_back(m.name);
      count.push_back(0);
      total.push_back(0.0);
    }
    ++count[k];
    total[k] += ms;
  }
  for (const Mark& m : g_marks) {  // the report is taken: recycle the events
    g_free.push_back(m.a);
    g_free.push_back(m.b);
  }
  g_marks.clear();
  size_t w = (size_t)snprintf(buf, len, "{");
  for (size_t k = 0; k < names.size() && w < len; ++k)
    w += (size_t)snprintf(buf + w, len - w, "%s\"%s\": [%ld, %.6f]", k ? ", " : "", names[k],
                          count[k], total[k]);
  if (w < len) w += (size_t)snprintf(buf + w, len - w, "}");
  if (w >= len) return fail(EMX_ENOMEM, "buffer too small for the timing report");
  return EMX_OK;
}

}  // extern "C"
