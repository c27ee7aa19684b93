// Asynchronous Les Houches Event (LHE 3.0) export of generated events.
//
// Thesis, MadFlow chapter (unweighted event exporter): events are written as
// LHE 3.0 <event> records on a CPU thread separate from the device work, so
// that host I/O never stalls the GPU.  Here: lhe_write_events gathers the
// kept events of a batch on the device into per-event order, copies them
// into a pinned host buffer on the caller's stream and records an event; the
// writer thread waits for that event, formats the records and writes them.
// The caller's stream is never synchronised.  Pinned buffers are pooled and
// reused; they are released by lhe_close.
//
// Formatting: std::to_chars (17 significant digits), a batch split over up
// to eight threads and written in order.
//
// Record layout (Les Houches accord, LHE 3.0): an <init> block with the beams
// and one process; per event a line NUP IDPRUP XWGTUP SCALUP AQEDUP AQCDUP and
// one line per particle: IDUP ISTUP MOTHUP1 MOTHUP2 ICOLUP1 ICOLUP2 PUP1..PUP5
// VTIMUP SPINUP.  The two incoming partons are massless along +z and -z with
// E = sqrt_s/2 each (the partonic centre-of-mass frame of the generator);
// outgoing particles have mothers 1 and 2.  Colour flow is not computed (0 0)
// and helicities are unknown (9).  Numbers are written with 17 significant
// digits, so FP64 values read back exactly.
#include "common.h"

#include <algorithm>
#include <charconv>
#include <condition_variable>
#include <deque>
#include <math.h>
#include <mutex>
#include <stdio.h>
#include <string.h>
#include <string>
#include <thread>
#include <vector>

namespace vgx {

// staging[j][i][c] (c: E, px, py, pz) for kept event j = idx[j] of
// mom[c][i][n_total]
__global__ __launch_bounds__(256) void k_lhe_gather(int n_part, int64_t n_total, const double* __restrict__ mom,
                                                    const int64_t* __restrict__ idx, int64_t n_kept,
                                                    double* __restrict__ staging) {
  const int64_t total = n_kept * n_part * 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t j = t / (n_part * 4);
    const int r = (int)(t - j * n_part * 4);
    const int i = r >> 2, c = r & 3;
    const int64_t e = idx ? idx[j] : j;
    staging[t] = mom[((int64_t)c * n_part + i) * n_total + e];
  }
}

}  // namespace vgx

using namespace vgx;

namespace {

struct Job {
  double* host = nullptr;     // pinned, [n][n_part][4]
  size_t cap = 0;             // doubles
  bool pinned = true;
  hipEvent_t ready = nullptr; // null for host-side batches
  int64_t n = 0;
  int n_part = 0;
  int pdg_in[2] = {0, 0};
  std::vector<int> pdg_out;
  std::vector<double> masses;
  double sqrt_s = 0.0, weight = 0.0, scale = 0.0, aqed = 0.0, aqcd = 0.0;
  int proc = 0;
};

}  // namespace

struct vgx_lhe {
  FILE* f = nullptr;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<Job> queue;
  std::vector<Job> pool;  // pinned buffers ready for reuse
  bool closing = false;
  int64_t written = 0, queued = 0;
  int error = 0;
  std::string err;
};

namespace {

// " <v>" with 17 significant digits (the text of printf's %.16e)
inline void put_d(std::string& out, double v) {
  char b[40];
  const auto r = std::to_chars(b, b + sizeof b, v, std::chars_format::scientific, 16);
  out.push_back(' ');
  out.append(b, r.ptr);
}

inline void put_i(std::string& out, long long v) {
  char b[24];
  const auto r = std::to_chars(b, b + sizeof b, v);
  out.push_back(' ');
  out.append(b, r.ptr);
}

void put_particle(std::string& out, int pdg, int status, int m1, int m2, double px, double py, double pz, double e,
                  double mass) {
  put_i(out, pdg);
  put_i(out, status);
  put_i(out, m1);
  put_i(out, m2);
  out.append(" 0 0");
  put_d(out, px);
  put_d(out, py);
  put_d(out, pz);
  put_d(out, e);
  put_d(out, mass);
  out.append(" 0 9\n");
}

void put_event(std::string& out, const Job& J, int64_t j) {
  out.append("<event>\n");
  put_i(out, 2 + J.n_part);
  put_i(out, J.proc);
  put_d(out, J.weight);
  put_d(out, J.scale);
  put_d(out, J.aqed);
  put_d(out, J.aqcd);
  out.push_back('\n');
  const double h = 0.5 * J.sqrt_s;
  put_particle(out, J.pdg_in[0], -1, 0, 0, 0.0, 0.0, h, h, 0.0);
  put_particle(out, J.pdg_in[1], -1, 0, 0, 0.0, 0.0, -h, h, 0.0);
  const double* p = J.host + (size_t)j * J.n_part * 4;
  for (int i = 0; i < J.n_part; ++i) {
    const double* v = p + 4 * i;
    put_particle(out, J.pdg_out[i], 1, 1, 2, v[1], v[2], v[3], v[0], J.masses[i]);
  }
  out.append("</event>\n");
}

// Format a batch: contiguous slices of events on up to kFormatThreads
// threads, written in order.
constexpr int kFormatThreads = 8;
constexpr int64_t kEventsPerThread = 4096;

bool format_and_write(const Job& J, FILE* f) {
  const int64_t want = (J.n + kEventsPerThread - 1) / kEventsPerThread;
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int T = (int)std::max<int64_t>(1, std::min<int64_t>(want, std::min(kFormatThreads, hw)));
  std::vector<std::string> parts(T);
  auto work = [&](int t) {
    const int64_t lo = J.n * t / T, hi = J.n * (t + 1) / T;
    parts[t].reserve((size_t)(hi - lo) * (size_t)(J.n_part + 4) * 110);
    for (int64_t j = lo; j < hi; ++j) put_event(parts[t], J, j);
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < T; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto& th : pool) th.join();
  for (const std::string& s : parts)
    if (fwrite(s.data(), 1, s.size(), f) != s.size()) return false;
  return true;
}

void writer_loop(vgx_lhe* h) {
  for (;;) {
    Job J;
    {
      std::unique_lock<std::mutex> lk(h->mu);
      h->cv.wait(lk, [&] { return !h->queue.empty() || h->closing; });
      if (h->queue.empty()) return;
      J = std::move(h->queue.front());
      h->queue.pop_front();
    }
    bool ok = true;
    if (J.ready) ok = hipEventSynchronize(J.ready) == hipSuccess;
    if (ok) ok = format_and_write(J, h->f);
    std::lock_guard<std::mutex> lk(h->mu);
    if (!ok && !h->error) {
      h->error = 1;
      h->err = J.ready ? "lhe: device copy or file write failed" : "lhe: file write failed";
    }
    h->written += J.n;
    if (J.pinned) {
      J.pdg_out.clear();
      J.masses.clear();
      h->pool.push_back(std::move(J));
    } else {
      free(J.host);
    }
    h->cv_done.notify_all();
  }
}

}  // namespace

extern "C" vgx_status lhe_open(const char* path, const vgx_lhe_init* init, vgx_lhe** out) {
  VGX_CHECK(path && init && out, "lhe_open: null argument");
  *out = nullptr;
  FILE* f = fopen(path, "w");
  VGX_CHECK(f, "lhe_open: cannot open %s for writing", path);
  fprintf(f, "<LesHouchesEvents version=\"3.0\">\n<header>\n<generator name=\"vgx\"/>\n</header>\n<init>\n");
  fprintf(f, " %d %d %.16e %.16e %d %d %d %d %d 1\n", init->beam_id[0], init->beam_id[1], init->beam_energy[0],
          init->beam_energy[1], init->pdf_group[0], init->pdf_group[1], init->pdf_set[0], init->pdf_set[1],
          init->weight_mode);
  fprintf(f, " %.16e %.16e %.16e %d\n</init>\n", init->xsec, init->xsec_err, init->xmax, init->proc_id);
  if (ferror(f)) {
    fclose(f);
    set_error("lhe_open: write to %s failed", path);
    return VGX_EINVAL;
  }
  vgx_lhe* h = new vgx_lhe();
  h->f = f;
  h->th = std::thread(writer_loop, h);
  *out = h;
  return VGX_OK;
}

static vgx_status lhe_check_batch(vgx_lhe* h, int32_t n_part, const int32_t* pdg_in, const int32_t* pdg_out,
                                  const double* masses, double sqrt_s) {
  VGX_CHECK(h, "lhe: null writer");
  VGX_CHECK(n_part >= 1 && n_part <= VGX_MAX_PART, "lhe: n_part %d out of 1..%d", n_part, VGX_MAX_PART);
  VGX_CHECK(pdg_in && pdg_out && masses, "lhe: null host array");
  VGX_CHECK(sqrt_s > 0.0 && isfinite(sqrt_s), "lhe: sqrt_s must be positive and finite");
  std::lock_guard<std::mutex> lk(h->mu);
  if (h->error) {
    set_error("%s", h->err.c_str());
    return VGX_EINVAL;
  }
  return VGX_OK;
}

static void lhe_fill_meta(Job& J, int32_t n_part, const int32_t* pdg_in, const int32_t* pdg_out, const double* masses,
                          const vgx_lhe_event_info* info) {
  J.n_part = n_part;
  J.pdg_in[0] = pdg_in[0];
  J.pdg_in[1] = pdg_in[1];
  J.pdg_out.assign(pdg_out, pdg_out + n_part);
  J.masses.assign(masses, masses + n_part);
  J.sqrt_s = info->sqrt_s;
  J.weight = info->weight;
  J.scale = info->scale;
  J.aqed = info->aqed;
  J.aqcd = info->aqcd;
  J.proc = info->proc_id;
}

extern "C" vgx_status lhe_write_events(vgx_lhe* h, int32_t n_part, const int32_t* pdg_in, const int32_t* pdg_out,
                                       const double* masses, const vgx_lhe_event_info* info, int64_t n_total,
                                       const double* mom_dev, const int64_t* idx_dev, int64_t n_kept, void* stream) {
  VGX_CHECK(info, "lhe_write_events: null info");
  VGX_TRY(lhe_check_batch(h, n_part, pdg_in, pdg_out, masses, info->sqrt_s));
  VGX_CHECK(n_kept >= 0 && n_total >= 0 && (idx_dev || n_kept <= n_total),
            "lhe_write_events: bad counts n_kept=%lld n_total=%lld", (long long)n_kept, (long long)n_total);
  if (n_kept == 0) return VGX_OK;
  VGX_CHECK(mom_dev, "lhe_write_events: null device momenta");
  hipStream_t st = (hipStream_t)stream;
  const size_t need = (size_t)n_kept * n_part * 4;
  Job J;
  {  // a pooled pinned buffer large enough, else a new one
    std::lock_guard<std::mutex> lk(h->mu);
    for (size_t k = 0; k < h->pool.size(); ++k)
      if (h->pool[k].cap >= need) {
        J = std::move(h->pool[k]);
        h->pool.erase(h->pool.begin() + (long)k);
        break;
      }
  }
  if (!J.host) {
    VGX_HIP(hipHostMalloc((void**)&J.host, need * sizeof(double), hipHostMallocDefault));
    J.cap = need;
  }
  if (!J.ready) VGX_HIP(hipEventCreateWithFlags(&J.ready, hipEventDisableTiming));
  double* staging = nullptr;
  hipError_t e = hipMallocAsync((void**)&staging, need * sizeof(double), st);
  if (e == hipSuccess) {
    const int64_t want = ((int64_t)need + 255) / 256;
    const int grid = (int)(want < (int64_t)device_cus() * 8 ? want : (int64_t)device_cus() * 8);
    hipLaunchKernelGGL(k_lhe_gather, dim3(grid), dim3(256), 0, st, n_part, n_total, mom_dev, idx_dev, n_kept, staging);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(J.host, staging, need * sizeof(double), hipMemcpyDeviceToHost, st);
    hipError_t ef = hipFreeAsync(staging, st);
    if (e == hipSuccess) e = ef;
  }
  if (e == hipSuccess) e = hipEventRecord(J.ready, st);
  if (e != hipSuccess) {
    std::lock_guard<std::mutex> lk(h->mu);
    h->pool.push_back(std::move(J));
    return hip_fail(e, "lhe_write_events", __FILE__, __LINE__);
  }
  lhe_fill_meta(J, n_part, pdg_in, pdg_out, masses, info);
  J.n = n_kept;
  std::lock_guard<std::mutex> lk(h->mu);
  h->queued += n_kept;
  h->queue.push_back(std::move(J));
  h->cv.notify_one();
  return VGX_OK;
}

extern "C" vgx_status lhe_write_events_host(vgx_lhe* h, int32_t n_part, const int32_t* pdg_in, const int32_t* pdg_out,
                                            const double* masses, const vgx_lhe_event_info* info, int64_t n,
                                            const double* mom_host) {
  VGX_CHECK(info, "lhe_write_events_host: null info");
  VGX_TRY(lhe_check_batch(h, n_part, pdg_in, pdg_out, masses, info->sqrt_s));
  VGX_CHECK(n >= 0, "lhe_write_events_host: n < 0");
  if (n == 0) return VGX_OK;
  VGX_CHECK(mom_host, "lhe_write_events_host: null momenta");
  Job J;
  J.pinned = false;
  J.cap = (size_t)n * n_part * 4;
  J.host = (double*)malloc(J.cap * sizeof(double));
  VGX_CHECK(J.host, "lhe_write_events_host: host allocation failed");
  memcpy(J.host, mom_host, J.cap * sizeof(double));
  lhe_fill_meta(J, n_part, pdg_in, pdg_out, masses, info);
  J.n = n;
  std::lock_guard<std::mutex> lk(h->mu);
  h->queued += n;
  h->queue.push_back(std::move(J));
  h->cv.notify_one();
  return VGX_OK;
}

extern "C" vgx_status lhe_flush(vgx_lhe* h, int64_t* written) {
  VGX_CHECK(h, "lhe_flush: null writer");
  std::unique_lock<std::mutex> lk(h->mu);
  h->cv_done.wait(lk, [&] { return h->written == h->queued; });
  if (written) *written = h->written;
  fflush(h->f);
  if (h->error) {
    set_error("%s", h->err.c_str());
    return VGX_EINVAL;
  }
  return VGX_OK;
}

extern "C" vgx_status lhe_close(vgx_lhe* h) {
  if (!h) return VGX_OK;
  {
    std::lock_guard<std::mutex> lk(h->mu);
    h->closing = true;
    h->cv.notify_all();
  }
  h->th.join();
  fprintf(h->f, "</LesHouchesEvents>\n");
  const bool bad = ferror(h->f) != 0;
  const int cl = fclose(h->f);
  const int error = h->error;
  std::string err = h->err;
  for (Job& J : h->pool) {
    if (J.host) hipHostFree(J.host);
    if (J.ready) hipEventDestroy(J.ready);
  }
  delete h;
  if (error) {
    set_error("%s", err.c_str());
    return VGX_EINVAL;
  }
  if (bad || cl != 0) {
    set_error("lhe_close: write failed");
    return VGX_EINVAL;
  }
  return VGX_OK;
}
