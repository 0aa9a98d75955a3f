// Resource monitor of a workload on one MI355X: the MI355X analogue of the
// paper's GPU monitor (Section 2: start a sampler, mark code phases with
// timestamps, stop, parse) together with its CPU monitor of the workload's
// process (Section 3.2).  Host code only.
//
// A sampler thread wakes every `period` seconds (on a fixed grid from the
// start, so the period does not drift) and appends one CSV row: the GPU's
// graphics and memory-controller activity, VRAM in use and in total, edge /
// hotspot / VRAM temperatures and socket power from amd-smi, and the
// monitored process's CPU share over the last period and resident memory
// from /proc, and the device memory in use as the HIP runtime reports it
// (total - free).  amd-smi is loaded at run time (dlopen), so the library
// does not depend on it; without it, or without a GPU, the GPU columns are
// NaN.
// Timestamps go to a second CSV as (time, name) rows, framed by "start" at 0
// and "stop" at the end; tsne_monitor_steps turns both into the step table
// (each interval between consecutive timestamps assigned to the first).
#include <amd_smi/amdsmi.h>
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <unistd.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "tsne_mi355x.h"

namespace tsne {
namespace mon {

using Clock = std::chrono::steady_clock;
constexpr double NaN = NAN;

// The amd-smi entry points used, resolved from the shared library.
struct Smi {
  void* lib = nullptr;
  decltype(&amdsmi_init) init = nullptr;
  decltype(&amdsmi_shut_down) shut_down = nullptr;
  decltype(&amdsmi_get_socket_handles) sockets = nullptr;
  decltype(&amdsmi_get_processor_handles) processors = nullptr;
  decltype(&amdsmi_get_gpu_device_bdf) bdf = nullptr;
  decltype(&amdsmi_get_gpu_activity) activity = nullptr;
  decltype(&amdsmi_get_gpu_memory_usage) mem_used = nullptr;
  decltype(&amdsmi_get_gpu_memory_total) mem_total = nullptr;
  decltype(&amdsmi_get_temp_metric) temp = nullptr;
  decltype(&amdsmi_get_power_info) power = nullptr;
  decltype(&amdsmi_get_gpu_vram_usage) vram = nullptr;
  amdsmi_processor_handle gpu = nullptr;
  bool inited = false;

  template <typename F>
  bool sym(F& f, const char* name) {
    f = reinterpret_cast<F>(dlsym(lib, name));
    return f != nullptr;
  }

  // The amd-smi processor whose PCI address is that of HIP device `dev`.
  bool open(int dev) {
    if (dev < 0) return false;
    int bus = -1, device = -1, domain = -1;
    if (hipDeviceGetAttribute(&bus, hipDeviceAttributePciBusId, dev) != hipSuccess ||
        hipDeviceGetAttribute(&device, hipDeviceAttributePciDeviceId, dev) != hipSuccess ||
        hipDeviceGetAttribute(&domain, hipDeviceAttributePciDomainId, dev) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    lib = dlopen("libamd_smi.so", RTLD_NOW | RTLD_LOCAL);
    if (!lib) lib = dlopen("/opt/rocm/lib/libamd_smi.so", RTLD_NOW | RTLD_LOCAL);
    if (!lib) return false;
    if (!(sym(init, "amdsmi_init") && sym(shut_down, "amdsmi_shut_down") && sym(sockets, "amdsmi_get_socket_handles") &&
          sym(processors, "amdsmi_get_processor_handles") && sym(bdf, "amdsmi_get_gpu_device_bdf") &&
          sym(activity, "amdsmi_get_gpu_activity") && sym(mem_used, "amdsmi_get_gpu_memory_usage") &&
          sym(mem_total, "amdsmi_get_gpu_memory_total") && sym(temp, "amdsmi_get_temp_metric") &&
          sym(power, "amdsmi_get_power_info")))
      return false;
    sym(vram, "amdsmi_get_gpu_vram_usage");  // optional
    if (init(AMDSMI_INIT_AMD_GPUS) != AMDSMI_STATUS_SUCCESS) return false;
    inited = true;
    uint32_t ns = 0;
    if (sockets(&ns, nullptr) != AMDSMI_STATUS_SUCCESS || ns == 0) return false;
    std::vector<amdsmi_socket_handle> sh(ns);
    if (sockets(&ns, sh.data()) != AMDSMI_STATUS_SUCCESS) return false;
    for (uint32_t s = 0; s < ns && !gpu; ++s) {
      uint32_t np = 0;
      if (processors(sh[s], &np, nullptr) != AMDSMI_STATUS_SUCCESS || np == 0) continue;
      std::vector<amdsmi_processor_handle> ph(np);
      if (processors(sh[s], &np, ph.data()) != AMDSMI_STATUS_SUCCESS) continue;
      for (uint32_t p = 0; p < np; ++p) {
        amdsmi_bdf_t b;
        if (bdf(ph[p], &b) != AMDSMI_STATUS_SUCCESS) continue;
        if (int(b.bus_number) == bus && int(b.device_number) == device && int64_t(b.domain_number) == domain) {
          gpu = ph[p];
          break;
        }
      }
    }
    return gpu != nullptr;
  }

  void close() {
    if (inited && shut_down) shut_down();
    if (lib) dlclose(lib);
    lib = nullptr;
    inited = false;
    gpu = nullptr;
  }
};

// /proc/<pid>/stat utime + stime in seconds, and /proc/<pid>/statm resident
// pages in bytes; NaN when unreadable.
double proc_cpu_seconds(int pid) {
  char path[64];
  std::snprintf(path, sizeof path, pid > 0 ? "/proc/%d/stat" : "/proc/self/stat", pid);
  FILE* f = std::fopen(path, "r");
  if (!f) return NaN;
  char buf[2048];
  const size_t len = std::fread(buf, 1, sizeof buf - 1, f);
  std::fclose(f);
  buf[len] = 0;
  const char* p = std::strrchr(buf, ')');  // the command name may hold spaces
  if (!p) return NaN;
  unsigned long long ut = 0, st = 0;
  // after ") ": state is field 3; utime and stime are fields 14 and 15
  if (std::sscanf(p + 2, "%*c %*d %*d %*d %*d %*d %*u %*u %*u %*u %*u %llu %llu", &ut, &st) != 2) return NaN;
  return double(ut + st) / double(sysconf(_SC_CLK_TCK));
}

double proc_rss_bytes(int pid) {
  char path[64];
  std::snprintf(path, sizeof path, pid > 0 ? "/proc/%d/statm" : "/proc/self/statm", pid);
  FILE* f = std::fopen(path, "r");
  if (!f) return NaN;
  unsigned long long size = 0, res = 0;
  const int got = std::fscanf(f, "%llu %llu", &size, &res);
  std::fclose(f);
  return got == 2 ? double(res) * double(sysconf(_SC_PAGESIZE)) : NaN;
}

const char* kHeader =
    "t_s,gfx_pct,umc_pct,vram_used_bytes,vram_total_bytes,temp_edge_c,temp_hotspot_c,temp_vram_c,power_w,"
    "proc_cpu_pct,proc_rss_bytes,hip_used_bytes,sample_us\n";

}  // namespace mon
}  // namespace tsne

struct tsne_monitor {
  tsne::mon::Smi smi;
  bool have_gpu = false;
  int hip_device = -1;
  int pid = 0;
  double period = 1.0;
  FILE* samples = nullptr;
  FILE* events = nullptr;
  tsne::mon::Clock::time_point t0;
  std::mutex mu;  // guards the events file
  std::mutex cv_mu;
  std::condition_variable cv;
  std::atomic<bool> stopping{false};
  std::thread worker;
  double last_cpu = NAN;
  double last_t = 0.0;

  double now() const { return std::chrono::duration<double>(tsne::mon::Clock::now() - t0).count(); }

  void sample() {
    using namespace tsne::mon;
    const auto a = Clock::now();
    double gfx = NaN, umc = NaN, used = NaN, total = NaN, te = NaN, th = NaN, tv = NaN, pw = NaN;
    if (have_gpu) {
      amdsmi_engine_usage_t u;
      if (smi.activity(smi.gpu, &u) == AMDSMI_STATUS_SUCCESS) {
        if (u.gfx_activity != UINT32_MAX) gfx = u.gfx_activity;
        if (u.umc_activity != UINT32_MAX) umc = u.umc_activity;
      }
      uint64_t v = 0;
      amdsmi_vram_usage_t vu;
      if (smi.vram && smi.vram(smi.gpu, &vu) == AMDSMI_STATUS_SUCCESS && vu.vram_used > 0)
        used = double(vu.vram_used) * 1048576.0;
      else if (smi.mem_used(smi.gpu, AMDSMI_MEM_TYPE_VRAM, &v) == AMDSMI_STATUS_SUCCESS)
        used = double(v);
      if (smi.mem_total(smi.gpu, AMDSMI_MEM_TYPE_VRAM, &v) == AMDSMI_STATUS_SUCCESS) total = double(v);
      int64_t c = 0;
      if (smi.temp(smi.gpu, AMDSMI_TEMPERATURE_TYPE_EDGE, AMDSMI_TEMP_CURRENT, &c) == AMDSMI_STATUS_SUCCESS) te = c;
      if (smi.temp(smi.gpu, AMDSMI_TEMPERATURE_TYPE_HOTSPOT, AMDSMI_TEMP_CURRENT, &c) == AMDSMI_STATUS_SUCCESS) th = c;
      if (smi.temp(smi.gpu, AMDSMI_TEMPERATURE_TYPE_VRAM, AMDSMI_TEMP_CURRENT, &c) == AMDSMI_STATUS_SUCCESS) tv = c;
      amdsmi_power_info_t p;
      if (smi.power(smi.gpu, &p) == AMDSMI_STATUS_SUCCESS) {
        if (p.current_socket_power != UINT32_MAX && p.current_socket_power != 0) pw = p.current_socket_power;
        else if (p.average_socket_power != UINT32_MAX) pw = p.average_socket_power;
      }
    }
    const double cpu_s = proc_cpu_seconds(pid);
    const double rss = proc_rss_bytes(pid);
    double hip_used = NaN;
    size_t fr = 0, tot = 0;
    if (hip_device >= 0 && hipMemGetInfo(&fr, &tot) == hipSuccess) hip_used = double(tot - fr);
    // the row's time is taken after its last reading: every reading in a row
    // precedes the row's time, so a row is never counted in the step before
    // a change it already shows
    const double t = now();
    double cpu_pct = NaN;
    if (std::isfinite(cpu_s) && std::isfinite(last_cpu) && t > last_t) cpu_pct = 100.0 * (cpu_s - last_cpu) / (t - last_t);
    last_cpu = cpu_s;
    last_t = t;
    const double us = std::chrono::duration<double, std::micro>(Clock::now() - a).count();
    std::fprintf(samples, "%.6f,%.17g,%.17g,%.17g,%.17g,%.17g,%.17g,%.17g,%.17g,%.17g,%.17g,%.17g,%.3f\n", t, gfx, umc,
                 used, total, te, th, tv, pw, cpu_pct, rss, hip_used, us);
    std::fflush(samples);
  }

  void run() {
    if (hip_device >= 0 && hipSetDevice(hip_device) != hipSuccess) {  // this thread's device for hipMemGetInfo
      (void)hipGetLastError();
      hip_device = -1;
    }
    int64_t k = 0;
    while (!stopping.load()) {
      sample();
      ++k;
      const auto next = t0 + std::chrono::duration_cast<tsne::mon::Clock::duration>(
                                 std::chrono::duration<double>(double(k) * period));
      std::unique_lock<std::mutex> lk(cv_mu);
      cv.wait_until(lk, next, [&] { return stopping.load(); });
    }
    sample();  // the state at stop
  }

  void event(const char* name) {
    std::string s(name);
    for (char& c : s)
      if (c == ',' || c == '\n' || c == '\r' || c == '"') c = '_';
    std::lock_guard<std::mutex> g(mu);
    std::fprintf(events, "%.6f,%s\n", now(), s.c_str());
    std::fflush(events);
  }
};

extern "C" int tsne_monitor_start(double period_s, int32_t hip_device, int32_t pid, const char* samples_csv,
                                  const char* events_csv, tsne_monitor** out) {
  if (!out || !samples_csv || !events_csv || !(period_s >= 1e-3) || !(period_s <= 3600.0) || pid < 0)
    return TSNE_ERR_INVALID_ARG;
  *out = nullptr;
  tsne_monitor* m = new (std::nothrow) tsne_monitor();
  if (!m) return TSNE_ERR_INVALID_ARG;
  m->period = period_s;
  m->pid = pid;
  m->samples = std::fopen(samples_csv, "w");
  m->events = m->samples ? std::fopen(events_csv, "w") : nullptr;
  if (!m->samples || !m->events) {
    if (m->samples) std::fclose(m->samples);
    delete m;
    return TSNE_ERR_INVALID_ARG;
  }
  m->have_gpu = m->smi.open(hip_device);
  int ndev = 0;
  if (hip_device >= 0 && hipGetDeviceCount(&ndev) == hipSuccess && hip_device < ndev) m->hip_device = hip_device;
  (void)hipGetLastError();
  std::fputs(tsne::mon::kHeader, m->samples);
  std::fputs("t_s,name\n", m->events);
  m->t0 = tsne::mon::Clock::now();
  m->event("start");
  try {
    m->worker = std::thread([m] { m->run(); });
  } catch (...) {  // no thread to be had: no exception crosses the ABI
    std::fclose(m->samples);
    std::fclose(m->events);
    m->smi.close();
    delete m;
    return TSNE_ERR_INVALID_ARG;
  }
  *out = m;
  return TSNE_OK;
}

extern "C" int tsne_monitor_timestamp(tsne_monitor* m, const char* name) {
  if (!m || !name) return TSNE_ERR_INVALID_ARG;
  m->event(name);
  return TSNE_OK;
}

extern "C" int tsne_monitor_has_gpu(const tsne_monitor* m) { return m && m->have_gpu ? 1 : 0; }

extern "C" int tsne_monitor_stop(tsne_monitor* m) {
  if (!m) return TSNE_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(m->cv_mu);
    m->stopping.store(true);
  }
  m->cv.notify_all();
  m->worker.join();
  m->event("stop");
  std::fclose(m->samples);
  std::fclose(m->events);
  m->smi.close();
  delete m;
  return TSNE_OK;
}

extern "C" int tsne_monitor_steps(const double* t, const double* values, int64_t n, int32_t n_fields,
                                  const double* events, int64_t n_events, int64_t* count, double* mean,
                                  double* maxv) {
  if (n < 0 || n_fields < 1 || n_events < 2 || !events || !count || !mean || !maxv || (n > 0 && (!t || !values)))
    return TSNE_ERR_INVALID_ARG;
  for (int64_t i = 1; i < n; ++i)
    if (!(t[i] >= t[i - 1])) return TSNE_ERR_INVALID_ARG;
  for (int64_t k = 1; k < n_events; ++k)
    if (!(events[k] >= events[k - 1])) return TSNE_ERR_INVALID_ARG;
  // samples ascending: one pass, each sample to the step whose interval
  // [events[k], events[k + 1]) holds it
  const int64_t ns = n_events - 1;
  std::vector<double> sum(size_t(ns) * n_fields, 0.0), mx(size_t(ns) * n_fields, -INFINITY);
  std::vector<int64_t> fin(size_t(ns) * n_fields, 0);
  for (int64_t k = 0; k < ns; ++k) count[k] = 0;
  int64_t k = 0;
  for (int64_t i = 0; i < n; ++i) {
    while (k < ns && !(t[i] < events[k + 1])) ++k;
    if (k >= ns) break;
    if (t[i] < events[k]) continue;
    ++count[k];
    for (int32_t q = 0; q < n_fields; ++q) {
      const double v = values[i * n_fields + q];
      if (!std::isfinite(v)) continue;
      const size_t o = size_t(k) * n_fields + q;
      sum[o] += v;
      fin[o] += 1;
      mx[o] = v > mx[o] ? v : mx[o];
    }
  }
  for (size_t o = 0; o < sum.size(); ++o) {
    mean[o] = fin[o] ? sum[o] / double(fin[o]) : NAN;
    maxv[o] = fin[o] ? mx[o] : NAN;
  }
  return TSNE_OK;
}
