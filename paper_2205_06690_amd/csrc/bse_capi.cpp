// C-ABI of libbse: system state, batching of pair propagations, and the
// orchestration of the kernels in prop_kernels.hip / bse_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bse.h"
#include "bse_kernels.h"
#include "prop_kernels.h"
#include "clean_mfma.h"
#include "contract_mfma.h"
#include "host_math.h"

using namespace bse;
using bse_host::splitmix64_draw;
using bse_host::tridiag_lowest;

namespace {

thread_local std::string g_err;

struct Fail {
  bse_status st;
};

void fail(bse_status st, const std::string& msg) {
  g_err = msg;
  throw Fail{st};
}

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
      fail(BSE_ERR_OOM, std::string(what) + ": " + hipGetErrorString(e));
    fail(BSE_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
}
#define HIPC(x) hip_check((x), #x)

// device buffer with RAII
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void alloc(size_t n) {
    if (n <= bytes && p) return;
    release();
    if (n == 0) return;
    HIPC(hipMalloc(&p, n));
    bytes = n;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  ~DBuf() { release(); }
  template <typename X> X* as() const { return reinterpret_cast<X*>(p); }
};

struct Timer {
  struct Rec {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
  };
  bool on = false;
  int level = 0;   // 1: the propagation passes and the contractions; 2: every timed section
  std::map<std::string, Rec> recs;
  std::vector<std::string> order;
  hipStream_t st = nullptr;
  std::pair<hipEvent_t, hipEvent_t>* begin(const char* name, int lvl = 2) {
    auto* p = slot(name, lvl);
    if (p) HIPC(hipEventRecord(p->first, st));
    return p;
  }
  // the event pair of a timed section whose launch records the events itself
  std::pair<hipEvent_t, hipEvent_t>* slot(const char* name, int lvl = 2) {
    if (!on || lvl > level) return nullptr;
    auto it = recs.find(name);
    if (it == recs.end()) {
      order.push_back(name);
      it = recs.emplace(name, Rec{}).first;
    }
    Rec& r = it->second;
    if (r.used == r.ev.size()) {
      hipEvent_t a, b;
      HIPC(hipEventCreate(&a));
      HIPC(hipEventCreate(&b));
      r.ev.push_back({a, b});
    }
    return &r.ev[r.used++];
  }
  void end(std::pair<hipEvent_t, hipEvent_t>* p) {
    if (p) HIPC(hipEventRecord(p->second, st));
  }
  void reset() {
    for (auto& kv : recs) kv.second.used = 0;
  }
  ~Timer() {
    for (auto& kv : recs)
      for (auto& e : kv.second.ev) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
      }
  }
};

struct Tables {
  DBuf tw, kph, pf, ph, k2;
};

}  // namespace

// Device scratch of the allocation-free entry point: one array per GPU,
// loaded with the library's code object and held until the process ends.
// Host code must not pass `scratch` itself to a kernel (on the host the name
// stands for a host-side shadow); every use goes through the device address
// that hipGetSymbolAddress gives for the current device (scratch_dev).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[MAX_DEVICES] = {};

// Called with `dev` current (at system creation): records the device
// address of this device's copy of `scratch`, once per device.
void init_scratch(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) fail(BSE_ERR_ARG, "device ordinal above the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[dev]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    fail(BSE_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_dev[dev] = reinterpret_cast<double*>(p);
}

double* scratch_dev(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (dev >= 0 && dev < MAX_DEVICES) ? g_scratch_dev[dev] : nullptr;
}

}  // namespace

struct bse_system {
  bse_config cfg{};
  int n = 0;
  size_t ng = 0;
  double dv = 0;
  hipStream_t stream = nullptr;
  int L = 0;
  bool deterministic = false;
  std::vector<double> vext;
  Tables tf;
  Tables td;
  // orbitals
  int n_orb = 0;
  std::vector<double> eps;
  DBuf phi64;     // [n_orb][ng] FP64
  DBuf phi_occ32; // [n_occ][ng] FP32 (mixed)
  DBuf phih, phil, phith, phitl;  // bf16 hi/lo splits of phi_occ32, [n_occ][ng] and [ng][Sp]
  std::vector<int8_t> xi;
  bool signs_given = false;
  DBuf xi_d;
  DBuf eta0;      // [L][ng] FP64
  DBuf h0;        // [L][ng] complex T: unperturbed set at t = 0 (mid-step form)
  DBuf hbuf;      // [2][L][ng] complex T: unperturbed set, current and next step
  DBuf n0;        // [L]
  bool ready = false;
  // batch workspace
  int cap_b = 0;
  DBuf d, u, dens, wpol, q, rho64, work, work64, part, part32, gpart, coef, coefE, E, pq_d, flags;
  DBuf pscale;    // [B][3] row sums of q, then [B] per-pair scales of the packed Poisson solves
  DBuf normpart;  // partial norms of the unperturbed set (check at the cleaning steps)
  int nchunk = 0;
  // A / spectrum state
  int a_no = 0, a_nc = 0;
  DBuf wij;       // [n_ij][ng] FP64 W_ij of the valence pairs
  DBuf A_d;       // [(n_o n_c)^2] FP64
  DBuf f0_d;      // [n_o n_c][3] dipoles
  DBuf lz_V, lz_w, lz_c, lz_s;  // Lanczos basis and scratch
  DBuf ba_pq, ba_X, ba_Dm, ba_part, ba_rho64, ba_v64, ba_cpart, ba_ev, ba_ec, ba_s[4];  // bse_build_A scratch
  Timer timer;
  int lz_path = 0;   // 0 fused launches where A fits, 1 a launch per operation
  std::vector<double> wts;
  int tune_tc = 0, tune_nt = 0;   // autotuned x-tile width / plane block size (0 = default)
  int launch_order = 5;           // workgroup order bits: x (1), y-line (2), fused y-z (4) passes (bse_set_launch_order)
  int yz_schedule = 2;            // where available: 2 plane pass, 16-point DFTs per lane; 0 cross-lane; 1 line passes
  hipStream_t own_stream = nullptr;
  // surrogate descriptors and buffers
  DBuf n0dens, vdev, fx, fy, fscale, fdots, fwpol;
  DBuf mx_f, mx_tf, mx_out, mx_rho, mx_dv, mx_c, mx_part, mx_eps;  // matrix-free A f
  int mx_eps_v0 = -1, mx_eps_n = 0;   // valence window whose eps mx_eps holds
  DBuf bnd_n, bnd_v, bnd_part;   // boundary potential: density, v_H, block sums
  double n0_scale = 0, v_scale = 0;
};

namespace {

int wsize(const bse_system* s) { return s->cfg.precision == BSE_FP64 ? 8 : 4; }

template <typename T>
void upload_tables(bse_system* s, Tables& tb) {
  using C = cplx<T>;
  const int n = s->n;
  const double h = s->cfg.h, dt = s->cfg.dt;
  std::vector<C> tw(n), kph(n);
  std::vector<T> k2(n);
  for (int m = 0; m < n; ++m) {
    const double a = -2.0 * M_PI * m / n;
    tw[m].x = (T)std::cos(a);
    tw[m].y = (T)std::sin(a);
    const int mm = (m < (n + 1) / 2) ? m : m - n;  // fftfreq ordering, Nyquist negative
    const double k = 2.0 * M_PI * mm / (n * h);
    k2[m] = (T)(k * k);
    const double ph = -0.5 * k * k * dt;
    kph[m].x = (T)(std::cos(ph) / n);
    kph[m].y = (T)(std::sin(ph) / n);
  }
  std::vector<C> pf(s->ng), phh(s->ng);
  for (size_t i = 0; i < s->ng; ++i) {
    const double v = s->vext[i];
    pf[i].x = (T)std::cos(-v * dt);
    pf[i].y = (T)std::sin(-v * dt);
    phh[i].x = (T)std::cos(-0.5 * v * dt);
    phh[i].y = (T)std::sin(-0.5 * v * dt);
  }
  tb.tw.alloc(sizeof(C) * n);
  tb.kph.alloc(sizeof(C) * n);
  tb.k2.alloc(sizeof(T) * n);
  tb.pf.alloc(sizeof(C) * s->ng);
  tb.ph.alloc(sizeof(C) * s->ng);
  HIPC(hipMemcpy(tb.tw.p, tw.data(), sizeof(C) * n, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(tb.kph.p, kph.data(), sizeof(C) * n, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(tb.k2.p, k2.data(), sizeof(T) * n, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(tb.pf.p, pf.data(), sizeof(C) * s->ng, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(tb.ph.p, phh.data(), sizeof(C) * s->ng, hipMemcpyHostToDevice));
}

template <typename T> Tables& tabs(bse_system* s);
template <> Tables& tabs<float>(bse_system* s) { return s->tf; }
template <> Tables& tabs<double>(bse_system* s) { return s->td; }

// Coulomb potential of B real FP64 densities (rho64) into q (FP64)
void poisson64(bse_system* s, const double* rho, int B, double* out, double* acc, double wn,
               int* flags = nullptr) {
  const size_t need = sizeof(cplx<double>) * s->ng * (size_t)((B + 1) / 2);
  s->work64.alloc(need);
  PoisArgs<double> a{};
  a.flags = flags;
  a.rho = rho;
  a.B = B;
  a.work = s->work64.as<cplx<double>>();
  a.tw = s->td.tw.as<cplx<double>>();
  a.k2 = s->td.k2.as<double>();
  a.vscale = 4.0 * M_PI / (double)s->ng;
  a.out64 = out;
  a.acc = acc;
  a.wn = wn;
  HIPC(launch_poisson<double>(s->n, a, s->stream));
}

template <typename T>
void ensure_batch(bse_system* s, int B) {
  using C = cplx<T>;
  if (B <= s->cap_b) return;
  const size_t ng = s->ng;
  const int L = s->L;
  const int S = s->cfg.n_occ;
  s->d.alloc(sizeof(C) * ng * (size_t)B * L);
  s->u.alloc(sizeof(T) * ng * B);
  s->dens.alloc(sizeof(T) * ng * B);
  s->wpol.alloc(sizeof(double) * ng * B);
  s->q.alloc(sizeof(double) * ng * B);
  s->rho64.alloc(sizeof(double) * ng * B);
  s->work.alloc(sizeof(C) * ng * (size_t)((B + 1) / 2));
  s->E.alloc(sizeof(C) * ng * L);
  const int chunk = 4096;
  s->nchunk = (int)((ng + chunk - 1) / chunk);
  const int F = B * L;
  s->part.alloc(sizeof(cplx<double>) * (size_t)s->nchunk * std::max(F, L) * (S + 1));
  s->coef.alloc(sizeof(cplx<double>) * (size_t)F * (S + 1));
  if (sizeof(T) == 4) {
    s->part32.alloc(sizeof(float) * clean_scratch_floats(F, L, S, ng));
    s->gpart.alloc(sizeof(cplx<double>) * edot_part_entries(F, L, S, ng));
  }
  s->coefE.alloc(sizeof(cplx<double>) * (size_t)L * (S + 1));
  s->pq_d.alloc(sizeof(int) * 2 * B);
  s->flags.alloc(sizeof(int) * B);
  s->work64.alloc(sizeof(cplx<double>) * ng * (size_t)((B + 1) / 2));
  s->pscale.alloc(sizeof(double) * 4 * (size_t)B);
  s->normpart.alloc(sizeof(double) * norm_drift_part_elems(L));
  s->cap_b = B;
}

template <typename T>
const T* occ_phi(bse_system* s);
template <> const float* occ_phi<float>(bse_system* s) { return s->phi_occ32.as<float>(); }
template <> const double* occ_phi<double>(bse_system* s) { return s->phi64.as<double>(); }

template <typename T>
void clean(bse_system* s, int B, int from_mid, const cplx<T>* H) {
  Tables& tb = tabs<T>(s);
  CleanArgs<T> c{};
  c.d = s->d.as<cplx<T>>();
  c.F = B * s->L;
  c.L = s->L;
  c.S = s->cfg.n_occ;
  c.u = s->u.as<T>();
  c.H = H;
  c.ph = tb.ph.as<cplx<T>>();
  c.E = s->E.as<cplx<T>>();
  c.phi = occ_phi<T>(s);
  c.ng = s->ng;
  c.dt = (T)s->cfg.dt;
  c.from_mid = from_mid;
  c.chunk = 4096;
  c.part = s->part.as<cplx<double>>();
  c.coef = s->coef.as<cplx<double>>();
  c.coefE = s->coefE.as<cplx<double>>();
  c.n0 = s->n0.as<double>();
  c.renorm = 1;
  c.dv = s->dv;
  c.dens = s->dens.as<T>();
  c.eta0 = s->eta0.as<double>();
  c.part32 = s->part32.as<float>();
  c.gpart = s->gpart.as<cplx<double>>();
  c.phih = s->phih.as<unsigned short>();
  c.phil = s->phil.as<unsigned short>();
  c.phith = s->phith.as<unsigned short>();
  c.phitl = s->phitl.as<unsigned short>();
  auto* t = s->timer.begin("clean");
  HIPC(launch_clean<T>(c, s->stream));
  s->timer.end(t);
}

template <typename T>
void poissonT(bse_system* s, int B, double* acc, double wn) {
  Tables& tb = tabs<T>(s);
  PoisArgs<T> a{};
  a.rho = s->dens.as<T>();
  a.B = B;
  a.work = s->work.as<cplx<T>>();
  a.tw = tb.tw.as<cplx<T>>();
  a.k2 = tb.k2.as<T>();
  a.vscale = (T)(4.0 * M_PI / (double)s->ng);
  a.out = s->u.as<T>();
  a.acc = acc;
  a.wn = wn;
  a.pscale = s->pscale.as<double>() + 3 * (size_t)B;
  a.flags = s->flags.as<int>();
  auto* t = s->timer.begin("poisson");
  HIPC(launch_poisson<T>(s->n, a, s->stream));
  s->timer.end(t);
}

// One propagation of B pairs (pair list pq_dev[B][2] on the device) in
// phases, so that the time steps of several systems can be interleaved:
// results W^pol (FP64) in s->wpol, q in s->q.  Only kernel launches and
// device-to-device work are issued, so the sequence can be captured into a
// HIP graph.  The unperturbed set is propagated alongside, double-buffered:
// H_0 in s->h0, H_n in hbuf[n & 1] for n >= 1.
template <typename T>
struct PropRun {
  bse_system* s;
  int B;
  const int* pq_dev;
  const cplx<T>* hcur;   // H_n
  bool half;             // the state is an end-of-step state (t = 0 or just cleaned)
};

template <typename T>
cplx<T>* prop_hbuf(bse_system* s, int n) {
  return s->hbuf.as<cplx<T>>() + (size_t)(n & 1) * (size_t)s->L * s->ng;
}

template <typename T>
void prop_begin(PropRun<T>& r) {
  using C = cplx<T>;
  bse_system* s = r.s;
  const int B = r.B;
  const size_t ng = s->ng;
  const int L = s->L;
  const int F = B * L;
  const int M = s->cfg.clean_every;
  hipStream_t st = s->stream;
  // per-pair failure flags, sticky over the whole propagation: bit 0 a
  // non-finite density met by a Poisson solve, bit 1 a norm drift of the
  // unperturbed set at a cleaning step (every pair), and the final check
  // of W sets bit 0 too
  HIPC(launch_fill_zero(s->flags.p, sizeof(int) * B, st));
  HIPC(launch_pair_density(s->phi64.as<double>(), r.pq_dev, B, ng, s->rho64.as<double>(), st));
  poisson64(s, s->rho64.as<double>(), B, s->q.as<double>(), nullptr, 0.0, s->flags.as<int>());
  // per-pair scales for the packed Poisson solves of the induced densities:
  // the RMS of q_b (the response is linear in it), so that a pair whose
  // source is orders of magnitude weaker than its partner's is not buried
  // in the partner's rounding
  HIPC(launch_row_dots(s->q.as<double>(), nullptr, nullptr, B, ng, s->pscale.as<double>(), st));
  HIPC(launch_rms_scales(s->pscale.as<double>(), B, ng, s->pscale.as<double>() + 3 * (size_t)B, st));
  HIPC(launch_fill_zero(s->wpol.p, sizeof(double) * ng * B, st));
  HIPC(launch_fill_zero(s->u.p, sizeof(T) * ng * B, st));
  HIPC(launch_kick<T>(s->q.as<double>(), s->eta0.as<double>(), L, F, ng, s->d.as<C>(), st));
  r.hcur = s->h0.as<C>();
  if (M > 0) clean<T>(s, B, 2, r.hcur);
  // u_0 = 0: a phase kick does not change the density, so the t = 0 term
  // of the time integral vanishes.
  r.half = true;
}

// the y-z schedule of this system's plane passes
struct YZSched {
  bool fused;
  int order;
  int fused_kind;
};
template <typename T>
YZSched yz_sched(const bse_system* s) {
  YZSched y;
  y.fused = s->yz_schedule != 1 && prop_yz_fused<T>(s->n);
  // bit 1 orders the y-line pass, bit 2 the fused y-z pass
  y.order = (s->launch_order >> (y.fused ? 2 : 1)) & 1;
  y.fused_kind = y.fused ? (s->yz_schedule == 2 ? 2 : 1) : 0;
  return y;
}

// unperturbed set: one step, H_n -> H_{n+1}, on stream st
template <typename T>
void prop_unperturbed_step(PropRun<T>& r, int n, hipStream_t st) {
  using C = cplx<T>;
  bse_system* s = r.s;
  Tables& tb = tabs<T>(s);
  C* hnext = prop_hbuf<T>(s, n + 1);
  PropXArgs<T> pe{};
  pe.din = r.hcur;
  pe.dout = hnext;
  pe.pf = tb.pf.as<C>();
  pe.ph = tb.ph.as<C>();
  pe.tw = tb.tw.as<C>();
  pe.kph = tb.kph.as<C>();
  pe.dt = (T)s->cfg.dt;
  pe.L = s->L;
  pe.mode = PX_ETA0;
  pe.order = s->launch_order & 1;
  HIPC(launch_prop_x<T>(s->n, pe, s->L, st, s->tune_tc));
  const YZSched y = yz_sched<T>(s);
  PropYZArgs<T> pze{};
  pze.d = hnext;
  pze.tw = tb.tw.as<C>();
  pze.kph = tb.kph.as<C>();
  pze.L = s->L;
  pze.density = 0;
  pze.order = y.order;
  pze.fused = y.fused_kind;
  HIPC(launch_prop_yz<T>(s->n, pze, s->L, st, s->tune_nt));
}

// the perturbed set's two passes of step n (hcur = H_n, half as after step n - 1)
template <typename T>
PropXArgs<T> prop_pair_x_args(bse_system* s, const cplx<T>* hcur, bool half) {
  using C = cplx<T>;
  Tables& tb = tabs<T>(s);
  PropXArgs<T> px{};
  px.din = s->d.as<C>();
  px.dout = s->d.as<C>();
  px.pf = tb.pf.as<C>();
  px.ph = tb.ph.as<C>();
  px.u = s->u.as<T>();
  px.H = hcur;
  px.tw = tb.tw.as<C>();
  px.kph = tb.kph.as<C>();
  px.dt = (T)s->cfg.dt;
  px.L = s->L;
  px.mode = half ? PX_HALF : PX_FULL;
  px.order = s->launch_order & 1;
  return px;
}
template <typename T>
PropYZArgs<T> prop_pair_yz_args(bse_system* s, const cplx<T>* hnext) {
  using C = cplx<T>;
  Tables& tb = tabs<T>(s);
  const YZSched y = yz_sched<T>(s);
  PropYZArgs<T> pz{};
  pz.d = s->d.as<C>();
  pz.H = hnext;
  pz.tw = tb.tw.as<C>();
  pz.kph = tb.kph.as<C>();
  pz.dens = s->dens.as<T>();
  pz.L = s->L;
  pz.density = 1;
  pz.order = y.order;
  pz.fused = y.fused_kind;
  return pz;
}
// the unperturbed set's step n, then the perturbed set's two passes of step n
template <typename T>
void prop_pair_passes(PropRun<T>& r, int n) {
  bse_system* s = r.s;
  prop_unperturbed_step<T>(r, n, s->stream);
  const PropXArgs<T> px = prop_pair_x_args<T>(s, r.hcur, r.half);
  auto* t1 = s->timer.slot("prop_x", 1);
  const LaunchEvents e1{t1 ? t1->first : nullptr, t1 ? t1->second : nullptr};
  HIPC(launch_prop_x<T>(s->n, px, r.B, s->stream, s->tune_tc, t1 ? &e1 : nullptr));
  const PropYZArgs<T> pz = prop_pair_yz_args<T>(s, prop_hbuf<T>(s, n + 1));
  const YZSched y = yz_sched<T>(s);
  const bool split = !y.fused && prop_yz_split<T>(s->n);
  auto* t2 = s->timer.slot(split ? "prop_z" : "prop_yz", 1);
  auto* t3 = split ? s->timer.slot("prop_y", 1) : nullptr;
  const LaunchEvents e2{t2 ? t2->first : nullptr, t2 ? t2->second : nullptr};
  const LaunchEvents e3{t3 ? t3->first : nullptr, t3 ? t3->second : nullptr};
  HIPC(launch_prop_yz<T>(s->n, pz, r.B, s->stream, s->tune_nt, t2 ? &e2 : nullptr, t3 ? &e3 : nullptr));
}

// the rest of step n after the passes: the potential of the new density
// (and its time-integral term), the cleaning every M steps
template <typename T>
void prop_after_passes(PropRun<T>& r, int n) {
  bse_system* s = r.s;
  const int B = r.B;
  const int M = s->cfg.clean_every;
  cplx<T>* hnext = prop_hbuf<T>(s, n + 1);
  const bool do_clean = M > 0 && ((n + 1) % M == 0);
  const double wn = s->wts[n + 1];
  if (!do_clean) {
    poissonT<T>(s, B, s->wpol.as<double>(), wn);
    r.half = false;
  } else {
    poissonT<T>(s, B, nullptr, 0.0);
    clean<T>(s, B, 1, hnext);
    // the check point of Eq. 15: the unperturbed set must keep the norms
    // of eta_l(0) under the unitary propagation
    HIPC(launch_norm_drift<T>(hnext, s->L, s->ng, s->dv, s->n0.as<double>(), sizeof(T) == 4 ? 1e-3 : 1e-8,
                              s->flags.as<int>(), B, s->normpart.as<double>(), s->stream));
    poissonT<T>(s, B, s->wpol.as<double>(), wn);
    r.half = true;
  }
  r.hcur = hnext;
}

template <typename T>
void propagate_batch(bse_system* s, int B, const int* pq_dev) {
  PropRun<T> r{s, B, pq_dev, nullptr, true};
  prop_begin<T>(r);
  for (int n = 0; n < s->cfg.n_steps; ++n) {
    prop_pair_passes<T>(r, n);   // with the unperturbed set's step
    prop_after_passes<T>(r, n);
  }
}

// stochastic orbitals eta(0), their norms, and the t = 0 unperturbed state
template <typename T>
void prepare_unperturbed(bse_system* s) {
  using C = cplx<T>;
  Tables& tb = tabs<T>(s);
  const size_t ng = s->ng;
  const int L = s->L;
  const size_t hstride = (size_t)L * ng;
  s->h0.alloc(sizeof(C) * hstride);
  s->hbuf.alloc(sizeof(C) * hstride * 2);
  s->eta0.alloc(sizeof(double) * hstride);
  s->n0.alloc(sizeof(double) * L);
  if (!s->deterministic) {
    s->xi_d.alloc((size_t)L * s->cfg.n_occ);
    HIPC(hipMemcpy(s->xi_d.p, s->xi.data(), (size_t)L * s->cfg.n_occ, hipMemcpyHostToDevice));
  }
  HIPC(launch_stoch_orbitals<T>(s->phi64.as<double>(), s->xi_d.as<signed char>(), L, s->cfg.n_occ,
                                s->deterministic ? 1 : 0, ng, tb.ph.as<C>(), s->eta0.as<double>(),
                                s->h0.as<C>(), s->stream));
  HIPC(launch_norms(s->eta0.as<double>(), L, ng, s->dv, s->n0.as<double>(), s->stream));
}

void compute_weights(bse_system* s) {
  s->wts.assign(s->cfg.n_steps + 1, 0.0);
  bse_host::time_weights(s->cfg.n_steps, s->cfg.dt, s->cfg.gamma, s->wts.data());
}

void check_ready(bse_system* s) {
  if (!s) fail(BSE_ERR_ARG, "null system");
  if (!s->ready) fail(BSE_ERR_STATE, "bse_set_orbitals has not been called");
}

void check_pairs(const bse_system* s, int n_pairs, const int32_t* pq) {
  for (int k = 0; k < n_pairs; ++k)
    if (pq[2 * k] < 0 || pq[2 * k] >= s->n_orb || pq[2 * k + 1] < 0 || pq[2 * k + 1] >= s->n_orb)
      fail(BSE_ERR_ARG, "pair index out of range");
}

// Run W for n_pairs pairs (host list pq, already validated) into device
// outputs [n_pairs][ng], FP64 (w_f32 = false) or FP32.  A pair whose
// propagation met a non-finite value or whose unperturbed set drifted is
// NaN-filled on the device; status_host (nullable) receives the per-pair
// status, which costs one synchronisation per batch.
void apply_w_device(bse_system* s, int n_pairs, const int32_t* pq, void* w_dev, bool w_f32, double* wpol_dev,
                    int32_t* status_host) {
  check_ready(s);
  if (n_pairs < 0 || (n_pairs > 0 && (!pq || !w_dev))) fail(BSE_ERR_ARG, "bad pair arguments");
  check_pairs(s, n_pairs, pq);
  s->timer.st = s->stream;
  const int Bmax = std::max(1, s->cfg.max_batch);
  bool any_bad = false;
  for (int k0 = 0; k0 < n_pairs; k0 += Bmax) {
    const int B = std::min(Bmax, n_pairs - k0);
    if (s->cfg.precision == BSE_FP64) ensure_batch<double>(s, B);
    else ensure_batch<float>(s, B);
    HIPC(hipMemcpyAsync(s->pq_d.p, pq + 2 * k0, sizeof(int) * 2 * B, hipMemcpyHostToDevice, s->stream));
    if (s->cfg.precision == BSE_FP64) propagate_batch<double>(s, B, s->pq_d.as<int>());
    else propagate_batch<float>(s, B, s->pq_d.as<int>());
    const size_t off = (size_t)k0 * s->ng;
    const size_t cnt = (size_t)B * s->ng;
    // W = q + W^pol; the check reads the FP64 sum before any narrowing
    double* wsum = w_f32 ? s->rho64.as<double>() : reinterpret_cast<double*>(w_dev) + off;
    HIPC(launch_add(s->q.as<double>(), s->wpol.as<double>(), cnt, wsum, s->stream));
    HIPC(launch_finite_check(wsum, B, s->ng, s->flags.as<int>(), s->stream));
    if (w_f32) {
      float* wf = reinterpret_cast<float*>(w_dev) + off;
      HIPC(launch_add_f32(s->q.as<double>(), s->wpol.as<double>(), cnt, wf, s->stream));
      HIPC(launch_nan_flagged_f32(wf, B, s->ng, s->flags.as<int>(), s->stream));
    } else {
      HIPC(launch_nan_flagged(wsum, B, s->ng, s->flags.as<int>(), s->stream));
    }
    if (wpol_dev) {
      HIPC(hipMemcpyAsync(wpol_dev + off, s->wpol.p, sizeof(double) * cnt, hipMemcpyDeviceToDevice,
                          s->stream));
      HIPC(launch_nan_flagged(wpol_dev + off, B, s->ng, s->flags.as<int>(), s->stream));
    }
    if (status_host) {
      std::vector<int> fl(B);
      HIPC(hipMemcpyAsync(fl.data(), s->flags.p, sizeof(int) * B, hipMemcpyDeviceToHost, s->stream));
      HIPC(hipStreamSynchronize(s->stream));
      for (int b = 0; b < B; ++b) {
        status_host[k0 + b] = fl[b] ? BSE_ERR_NUMERIC : 0;
        if (fl[b]) any_bad = true;
      }
    }
  }
  if (any_bad) fail(BSE_ERR_NUMERIC, "non-finite W (or a drifting unperturbed set) for some pairs");
}

// ---------------------------------------------------------------------------
// Tamm-Dancoff matrix (Eq. 1)
// ---------------------------------------------------------------------------
void build_a(bse_system* s, int n_o, int n_c, double* A_host) {
  check_ready(s);
  const int n_occ = s->cfg.n_occ;
  if (n_o < 1 || n_o > n_occ || n_c < 1 || n_occ + n_c > s->n_orb || !A_host)
    fail(BSE_ERR_ARG, "bse_build_A: need 1 <= n_o <= n_occ and n_occ + n_c <= n_orb");
  const size_t ng = s->ng;
  const int v0 = n_occ - n_o, c0 = n_occ;
  const int n_ij = n_o * (n_o + 1) / 2, n_ia = n_o * n_c, n_ab = n_c * (n_c + 1) / 2;
  std::vector<int> pij, pia, pab;
  for (int i = 0; i < n_o; ++i)
    for (int j = i; j < n_o; ++j) { pij.push_back(v0 + i); pij.push_back(v0 + j); }
  for (int i = 0; i < n_o; ++i)
    for (int a = 0; a < n_c; ++a) { pia.push_back(v0 + i); pia.push_back(c0 + a); }
  for (int a = 0; a < n_c; ++a)
    for (int b = a; b < n_c; ++b) { pab.push_back(c0 + a); pab.push_back(c0 + b); }
  hipStream_t st = s->stream;
  // 1. W_ij for the valence pairs (kept on the device)
  s->wij.alloc(sizeof(double) * ng * n_ij);
  {
    std::vector<int32_t> stw(n_ij, 0);
    try {
      apply_w_device(s, n_ij, pij.data(), s->wij.as<double>(), false, nullptr, stw.data());
    } catch (const Fail& f) {
      if (f.st != BSE_ERR_NUMERIC) throw;
      int nb = 0;
      for (int k = 0; k < n_ij; ++k) nb += stw[k] != 0;
      fail(BSE_ERR_NUMERIC, "bse_build_A: W_ij failed the numerical checks for " + std::to_string(nb) + " of " +
                                std::to_string(n_ij) + " valence pairs");
    }
  }
  // scratch kept by the system across calls (grow-only), so repeated
  // builds allocate nothing
  DBuf& pq = s->ba_pq;
  pq.alloc(sizeof(int) * 2 * (size_t)std::max(std::max(n_ia, n_ab), n_ij));
  const bool fp64 = s->cfg.precision == BSE_FP64;
  DBuf &X = s->ba_X, &Dm = s->ba_Dm, &part = s->ba_part, &rho64 = s->ba_rho64, &v64 = s->ba_v64,
       &cpart = s->ba_cpart;
  // the buffers shared by the exchange and direct terms get their largest
  // size first, so that none is reallocated while kernels still use it
  if (fp64) {
    s->ba_s[0].alloc(sizeof(double) * ng * n_ab);
  } else {
    s->ba_s[0].alloc(sizeof(unsigned short) * ng * std::max(n_ia, n_ab));
    s->ba_s[1].alloc(sizeof(unsigned short) * ng * std::max(n_ia, n_ab));
    s->ba_s[2].alloc(sizeof(unsigned short) * ng * std::max(n_ia, n_ij));
    s->ba_s[3].alloc(sizeof(unsigned short) * ng * std::max(n_ia, n_ij));
    cpart.alloc(sizeof(float) * std::max(contract_part_floats(n_ia, n_ia, ng), contract_part_floats(n_ab, n_ij, ng)));
  }
  X.alloc(sizeof(double) * (size_t)n_ia * n_ia);
  Dm.alloc(sizeof(double) * (size_t)n_ab * n_ij);
  const size_t pe = std::max(gemm_part_elems(n_ia, n_ia, ng), gemm_part_elems(n_ab, n_ij, ng));
  if (fp64) part.alloc(pe * sizeof(double));
  // 2. exchange (ia|jb): Coulomb potentials of rho_jb in FP64, then the grid GEMM
  HIPC(hipMemcpyAsync(pq.p, pia.data(), sizeof(int) * 2 * n_ia, hipMemcpyHostToDevice, st));
  rho64.alloc(sizeof(double) * ng * n_ia);
  v64.alloc(sizeof(double) * ng * n_ia);
  HIPC(launch_products<double>(s->phi64.as<double>(), pq.as<int>(), n_ia, ng, rho64.as<double>(), st));
  const int PB = 64;
  for (int k0 = 0; k0 < n_ia; k0 += PB) {
    const int B = std::min(PB, n_ia - k0);
    poisson64(s, rho64.as<double>() + (size_t)k0 * ng, B, v64.as<double>() + (size_t)k0 * ng,
              nullptr, 0.0);
  }
  if (fp64) {
    HIPC(launch_gemm_f64(rho64.as<double>(), n_ia, v64.as<double>(), n_ia, ng, s->dv,
                         part.as<double>(), X.as<double>(), st));
  } else {
    // operands split once from FP64 into bf16 pairs for the matrix cores
    DBuf &rh = s->ba_s[0], &rl = s->ba_s[1], &vh = s->ba_s[2], &vl = s->ba_s[3];
    rh.alloc(sizeof(unsigned short) * ng * n_ia);
    rl.alloc(sizeof(unsigned short) * ng * n_ia);
    vh.alloc(sizeof(unsigned short) * ng * n_ia);
    vl.alloc(sizeof(unsigned short) * ng * n_ia);
    HIPC(launch_split64(rho64.as<double>(), ng * n_ia, rh.as<unsigned short>(), rl.as<unsigned short>(), st));
    HIPC(launch_split64(v64.as<double>(), ng * n_ia, vh.as<unsigned short>(), vl.as<unsigned short>(), st));
    cpart.alloc(sizeof(float) * contract_part_floats(n_ia, n_ia, ng));
    auto* t = s->timer.slot("gemm_exchange", 1);
    auto* tr = s->timer.slot("reduce_exchange", 1);
    const LaunchEvents e{t ? t->first : nullptr, t ? t->second : nullptr};
    const LaunchEvents er{tr ? tr->first : nullptr, tr ? tr->second : nullptr};
    HIPC(launch_contract_x3(rh.as<unsigned short>(), rl.as<unsigned short>(), n_ia, vh.as<unsigned short>(),
                            vl.as<unsigned short>(), n_ia, ng, s->dv, cpart.as<float>(), X.as<double>(), st,
                            t ? &e : nullptr, tr ? &er : nullptr));
  }
  // 3. direct (ab|W|ij) over a <= b and i <= j (pq is rewritten in stream order)
  HIPC(hipMemcpyAsync(pq.p, pab.data(), sizeof(int) * 2 * n_ab, hipMemcpyHostToDevice, st));
  if (fp64) {
    DBuf& rab = s->ba_s[0];
    rab.alloc(sizeof(double) * ng * n_ab);
    HIPC(launch_products<double>(s->phi64.as<double>(), pq.as<int>(), n_ab, ng, rab.as<double>(), st));
    HIPC(launch_gemm_f64(rab.as<double>(), n_ab, s->wij.as<double>(), n_ij, ng, s->dv,
                         part.as<double>(), Dm.as<double>(), st));
    HIPC(hipStreamSynchronize(st));
  } else {
    DBuf &abh = s->ba_s[0], &abl = s->ba_s[1], &wh = s->ba_s[2], &wl = s->ba_s[3];
    abh.alloc(sizeof(unsigned short) * ng * n_ab);
    abl.alloc(sizeof(unsigned short) * ng * n_ab);
    wh.alloc(sizeof(unsigned short) * ng * n_ij);
    wl.alloc(sizeof(unsigned short) * ng * n_ij);
    HIPC(launch_products_split(s->phi64.as<double>(), pq.as<int>(), n_ab, ng, abh.as<unsigned short>(),
                               abl.as<unsigned short>(), st));
    HIPC(launch_split64(s->wij.as<double>(), ng * n_ij, wh.as<unsigned short>(), wl.as<unsigned short>(), st));
    cpart.alloc(sizeof(float) * contract_part_floats(n_ab, n_ij, ng));
    auto* t = s->timer.slot("gemm_direct", 1);
    auto* tr = s->timer.slot("reduce_direct", 1);
    const LaunchEvents e{t ? t->first : nullptr, t ? t->second : nullptr};
    const LaunchEvents er{tr ? tr->first : nullptr, tr ? tr->second : nullptr};
    HIPC(launch_contract_x3(abh.as<unsigned short>(), abl.as<unsigned short>(), n_ab, wh.as<unsigned short>(),
                            wl.as<unsigned short>(), n_ij, ng, s->dv, cpart.as<float>(), Dm.as<double>(), st,
                            t ? &e : nullptr, tr ? &er : nullptr));
  }
  // 4. assemble
  DBuf &ev = s->ba_ev, &ec = s->ba_ec;
  ev.alloc(sizeof(double) * n_o);
  ec.alloc(sizeof(double) * n_c);
  HIPC(hipMemcpyAsync(ev.p, s->eps.data() + v0, sizeof(double) * n_o, hipMemcpyHostToDevice, st));
  HIPC(hipMemcpyAsync(ec.p, s->eps.data() + c0, sizeof(double) * n_c, hipMemcpyHostToDevice, st));
  s->A_d.alloc(sizeof(double) * (size_t)n_ia * n_ia);
  HIPC(launch_assemble_a(X.as<double>(), Dm.as<double>(), n_o, n_c, n_ij, ev.as<double>(),
                         ec.as<double>(), s->cfg.scissors, s->A_d.as<double>(), st));
  // dipoles of the transitions for the spectrum
  HIPC(hipMemcpyAsync(pq.p, pia.data(), sizeof(int) * 2 * n_ia, hipMemcpyHostToDevice, st));
  s->f0_d.alloc(sizeof(double) * 3 * n_ia);
  HIPC(launch_dipoles(s->phi64.as<double>(), pq.as<int>(), n_ia, s->n, s->cfg.h, s->f0_d.as<double>(), st));
  HIPC(hipMemcpyAsync(A_host, s->A_d.p, sizeof(double) * (size_t)n_ia * n_ia, hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  for (size_t k = 0; k < (size_t)n_ia * n_ia; ++k)
    if (!std::isfinite(A_host[k])) {
      s->a_no = s->a_nc = 0;   // no spectrum of a failed A
      fail(BSE_ERR_NUMERIC, "bse_build_A: non-finite element in A (exchange or direct term)");
    }
  s->a_no = n_o;
  s->a_nc = n_c;
}

// Lanczos with full re-orthogonalisation on the device copy of A.  The
// iterations run on the device without host round trips: the diagonal
// elements and squared residual norms stay in device arrays, and the host
// reads them only at the convergence checks (first at m = n_exc, then every
// 10 steps), where it also finds the first breakdown, if any.
void spectrum(bse_system* s, int n_exc, double* omega, double* dip2, int n_w, const double* w_grid,
              double sig, double* sigma) {
  if (!s) fail(BSE_ERR_ARG, "null system");
  if (s->a_no == 0) fail(BSE_ERR_STATE, "bse_spectrum: call bse_build_A first");
  const int n = s->a_no * s->a_nc;
  if (n_exc < 1 || n_exc > n || !omega || !dip2 || n_w < 0 || (n_w > 0 && (!w_grid || !sigma || !(sig > 0))))
    fail(BSE_ERR_ARG, "bse_spectrum: bad arguments");
  hipStream_t st = s->stream;
  s->lz_V.alloc(sizeof(double) * (size_t)(n + 1) * n);
  s->lz_w.alloc(sizeof(double) * (size_t)n * std::max(1, n_exc));
  s->lz_c.alloc(sizeof(double) * (n + 1));
  s->lz_s.alloc(sizeof(double) * ((size_t)n * n_exc + 2 * (size_t)n));
  double* V = s->lz_V.as<double>();
  double* w = s->lz_w.as<double>();
  double* c = s->lz_c.as<double>();
  double* al_d = s->lz_s.as<double>() + (size_t)n * n_exc;   // alpha_k
  double* bq_d = al_d + n;                                     // |w_k|^2
  // deterministic start vector (SplitMix64 draws in [-1, 1))
  std::vector<double> v0(n);
  double nr = 0;
  for (int i = 0; i < n; ++i) {
    v0[i] = (double)(splitmix64_draw(0x5EED5EEDULL, i) >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    nr += v0[i] * v0[i];
  }
  for (int i = 0; i < n; ++i) v0[i] /= std::sqrt(nr);
  HIPC(hipMemcpyAsync(V, v0.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
  std::vector<double> al(n), bq(n), alpha, beta;
  std::vector<double> theta;
  std::vector<std::vector<double>> svec;
  int m = 0, done = 0;
  const bool fused = s->lz_path == 0 && n <= lanczos_fused_max();
  for (int k = 0; k < n && !m; ++k) {
    const int mk = k + 1;
    const bool check = mk >= n_exc && ((mk - n_exc) % 10 == 0 || mk == n);
    if (fused) {
      // every iteration up to the next convergence check in one launch
      if (!check) continue;
      HIPC(launch_lanczos_steps(s->A_d.as<double>(), n, V, done, mk, al_d, bq_d, st));
    } else {
      HIPC(launch_gemv(s->A_d.as<double>(), n, V + (size_t)k * n, w, st));
      // two passes of classical Gram-Schmidt against the whole basis
      HIPC(launch_reorth(V, n, k + 1, c, w, st, al_d + k));
      HIPC(launch_reorth(V, n, k + 1, c, w, st));
      HIPC(launch_dot(w, w, n, bq_d + k, st));
      if (k + 1 < n) HIPC(launch_scale_norm(w, n, bq_d + k, V + (size_t)(k + 1) * n, st));
      if (!check) continue;
    }
    HIPC(hipMemcpyAsync(al.data() + done, al_d + done, sizeof(double) * (mk - done),
                        hipMemcpyDeviceToHost, st));
    HIPC(hipMemcpyAsync(bq.data() + done, bq_d + done, sizeof(double) * (mk - done),
                        hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    done = mk;
    // the recurrence in order: running norm estimate and first breakdown
    alpha.clear();
    beta.clear();
    double anorm = 0;
    int mm = mk;
    bool breakdown = false;
    for (int q = 0; q < mk; ++q) {
      const double b_q = std::sqrt(std::max(bq[q], 0.0));
      alpha.push_back(al[q]);
      anorm = std::max(anorm, std::fabs(al[q]) + b_q);
      if (b_q < 1e-13 * std::max(anorm, 1e-300)) {
        breakdown = true;
        mm = q + 1;
        break;
      }
      if (q + 1 < mk) beta.push_back(b_q);
    }
    if (mm < n_exc) fail(BSE_ERR_NUMERIC, "Lanczos subspace smaller than n_exc");
    // the convergence test takes Ritz values to 1e-9 (the last components of
    // their vectors barely depend on that); the final ones are resolved fully
    tridiag_lowest(alpha, beta, mm, std::min(n_exc, mm), theta, svec, 1e-9);
    const double b_last = std::sqrt(std::max(bq[mm - 1], 0.0));
    bool conv = true;
    for (int j = 0; j < (int)theta.size() && conv; ++j)
      if (b_last * std::fabs(svec[j][mm - 1]) > 1e-10 * std::max(anorm, 1.0)) conv = false;
    if (conv || breakdown || mk == n) {
      m = mm;
      tridiag_lowest(alpha, beta, mm, std::min(n_exc, mm), theta, svec);
    }
  }
  if (m == 0 || (int)theta.size() < n_exc) fail(BSE_ERR_NUMERIC, "Lanczos subspace smaller than n_exc");
  // Ritz vectors (all at once) and dipole strengths
  std::vector<double> f0(3 * (size_t)n), x((size_t)n * n_exc), sv((size_t)m * n_exc);
  for (int j = 0; j < n_exc; ++j)
    for (int q = 0; q < m; ++q) sv[(size_t)j * m + q] = svec[j][q];
  HIPC(hipMemcpyAsync(s->lz_s.p, sv.data(), sizeof(double) * sv.size(), hipMemcpyHostToDevice, st));
  HIPC(launch_ritz(V, n, m, s->lz_s.as<double>(), n_exc, w, st));
  HIPC(hipMemcpyAsync(x.data(), w, sizeof(double) * x.size(), hipMemcpyDeviceToHost, st));
  HIPC(hipMemcpyAsync(f0.data(), s->f0_d.p, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  for (int j = 0; j < n_exc; ++j) {
    omega[j] = theta[j];
    for (int ax = 0; ax < 3; ++ax) {
      double d = 0;
      for (int i = 0; i < n; ++i) d += x[(size_t)j * n + i] * f0[(size_t)i * 3 + ax];
      dip2[(size_t)j * 3 + ax] = d * d;
    }
  }
  for (int q = 0; q < n_w; ++q) {
    double acc = 0;
    for (int j = 0; j < n_exc; ++j) {
      const double z = (w_grid[q] - omega[j]) / sig;
      acc += (dip2[3 * j] + dip2[3 * j + 1] + dip2[3 * j + 2]) * std::exp(-0.5 * z * z);
    }
    sigma[q] = w_grid[q] * acc / (sig * std::sqrt(2.0 * M_PI));
  }
}

// Matrix-free A f in the mixed hole-grid representation (Eq. 6 with
// A = Q A-bar) for the valence window of the last bse_build_A, FP64: the
// kinetic term by the FFT pipeline with the k^2/2 multiplier, the Hartree
// term from dn = 2 sum phi_i f_i, the exchange-like term from the cached
// W_ij, then the occupied-space projection as a GEMM and an update.
// C[n_o][S] = dv sum_r f_i phi_s: the streaming projection kernel for up to
// 32 fields, the tiled FP64 GEMM beyond; part holds proj_scratch(n_o, S, ng)
size_t proj_scratch(int n_o, int S, size_t ng) {
  return n_o <= 32 ? proj_part_elems(n_o, S) : gemm_part_elems(n_o, S, ng);
}
void proj_coef(const double* f, int n_o, const double* phi, int S, size_t ng, double dv, double* part,
               double* C, hipStream_t st) {
  if (n_o <= 32) HIPC(launch_proj_coef(f, n_o, phi, S, ng, dv, part, C, st));
  else HIPC(launch_gemm_f64(f, n_o, phi, S, ng, dv, part, C, st));
}

void apply_a_mixed_device(bse_system* s, const double* f_dev, double* af_dev) {
  const int n_o = s->a_no, S = s->cfg.n_occ;
  const size_t ng = s->ng;
  hipStream_t st = s->stream;
  const double* phv = s->phi64.as<double>() + (size_t)(S - n_o) * ng;
  s->mx_tf.alloc(sizeof(double) * ng * n_o);
  s->mx_rho.alloc(sizeof(double) * ng);
  s->mx_dv.alloc(sizeof(double) * ng);
  s->mx_c.alloc(sizeof(double) * (size_t)n_o * S);
  s->mx_part.alloc(sizeof(double) * proj_scratch(n_o, S, ng));
  s->work64.alloc(sizeof(cplx<double>) * ng * (size_t)((n_o + 1) / 2));
  if (!s->vdev.p || s->vdev.bytes < sizeof(double) * ng) {
    s->vdev.alloc(sizeof(double) * ng);
    HIPC(hipMemcpy(s->vdev.p, s->vext.data(), sizeof(double) * ng, hipMemcpyHostToDevice));
  }
  if (s->mx_eps_v0 != S - n_o || s->mx_eps_n != n_o) {
    HIPC(hipStreamSynchronize(st));   // earlier applications may still read mx_eps
    s->mx_eps.alloc(sizeof(double) * n_o);
    HIPC(hipMemcpy(s->mx_eps.p, s->eps.data() + (S - n_o), sizeof(double) * n_o, hipMemcpyHostToDevice));
    s->mx_eps_v0 = S - n_o;
    s->mx_eps_n = n_o;
  }
  // kinetic term: T f_j for the n_o real fields (two per complex transform)
  PoisArgs<double> a{};
  a.rho = f_dev;
  a.B = n_o;
  a.work = s->work64.as<cplx<double>>();
  a.tw = s->td.tw.as<cplx<double>>();
  a.k2 = s->td.k2.as<double>();
  a.vscale = 1.0 / (double)ng;
  a.kinetic = 1;
  a.out64 = s->mx_tf.as<double>();
  HIPC(launch_poisson<double>(s->n, a, st));
  // Hartree term
  HIPC(launch_mixed_density(phv, f_dev, n_o, ng, s->mx_rho.as<double>(), st));
  poisson64(s, s->mx_rho.as<double>(), 1, s->mx_dv.as<double>(), nullptr, 0.0);
  HIPC(launch_mixed_combine(f_dev, s->mx_tf.as<double>(), s->vdev.as<double>(), s->mx_eps.as<double>(),
                            s->cfg.scissors, s->mx_dv.as<double>(), phv, s->wij.as<double>(), n_o, ng,
                            af_dev, st));
  // Q: coefficients on the occupied orbitals, then the update
  proj_coef(af_dev, n_o, s->phi64.as<double>(), S, ng, s->dv, s->mx_part.as<double>(), s->mx_c.as<double>(),
            st);
  HIPC(launch_project_out(af_dev, n_o, s->phi64.as<double>(), S, s->mx_c.as<double>(), ng, st));
}

void apply_a_mixed(bse_system* s, int n_vec, const double* f, double* af) {
  if (!s) fail(BSE_ERR_ARG, "null system");
  if (s->a_no == 0) fail(BSE_ERR_STATE, "bse_apply_A_mixed: call bse_build_A first");
  if (n_vec < 0 || (n_vec > 0 && (!f || !af))) fail(BSE_ERR_ARG, "bse_apply_A_mixed: bad arguments");
  if ((size_t)s->a_no * s->cfg.n_occ * sizeof(double) > 64 * 1024)
    fail(BSE_ERR_ARG, "bse_apply_A_mixed: n_o * n_occ above 8192");
  const size_t len = (size_t)s->a_no * s->ng;
  s->mx_f.alloc(sizeof(double) * len);
  s->mx_out.alloc(sizeof(double) * len);
  for (int v = 0; v < n_vec; ++v) {
    HIPC(hipMemcpyAsync(s->mx_f.p, f + v * len, sizeof(double) * len, hipMemcpyHostToDevice, s->stream));
    apply_a_mixed_device(s, s->mx_f.as<double>(), s->mx_out.as<double>());
    HIPC(hipMemcpyAsync(af + v * len, s->mx_out.p, sizeof(double) * len, hipMemcpyDeviceToHost, s->stream));
  }
  HIPC(hipStreamSynchronize(s->stream));
}

// The paper's spectrum algorithm (Eqs. 6-8): the Chebyshev recursion with A
// applied matrix-free in the mixed representation, from the dipole states
// f0_j = Q (r_axis - centre) phi_j of each axis; residues by the doubling
// identities, the spectrum as in chebyshev_spectrum.
void chebyshev_mixed(bse_system* s, int n_mom, double e_min, double e_max, int n_w,
                     const double* w_grid, double sig, double* sigma, double* residues) {
  if (!s) fail(BSE_ERR_ARG, "null system");
  if (s->a_no == 0) fail(BSE_ERR_STATE, "bse_chebyshev_mixed: call bse_build_A first");
  if (n_mom < 2 || n_mom % 2 != 0 || !(e_min < e_max) || n_w < 0 ||
      (n_w > 0 && (!w_grid || !sigma || !(sig > 0))) || (n_w == 0 && !residues))
    fail(BSE_ERR_ARG, "bse_chebyshev_mixed: bad arguments");
  if ((size_t)s->a_no * s->cfg.n_occ * sizeof(double) > 64 * 1024)
    fail(BSE_ERR_ARG, "bse_chebyshev_mixed: n_o * n_occ above 8192");
  hipStream_t st = s->stream;
  const int n_o = s->a_no, S = s->cfg.n_occ;
  const size_t ng = s->ng, len = (size_t)n_o * ng;
  const double b = 0.5 * (e_max + e_min), a = 0.5 * (e_max - e_min) * 1.01;
  const int K = n_mom / 2, nblk = mixed_cheb_blocks(), M = 2 * n_mom;
  DBuf fv, af, part, mu, D, wd, sd, cq, pq;
  fv.alloc(sizeof(double) * 9 * len);               // [pol][3 rotating vectors][n_o][ng]
  af.alloc(sizeof(double) * len);
  part.alloc(sizeof(double) * 6 * (size_t)K * nblk);
  mu.alloc(sizeof(double) * 3 * (size_t)n_mom);
  D.alloc(sizeof(double) * 3 * (size_t)M);
  cq.alloc(sizeof(double) * (size_t)n_o * S);
  pq.alloc(sizeof(double) * proj_scratch(n_o, S, ng));
  if (n_w > 0) {
    wd.alloc(sizeof(double) * n_w);
    sd.alloc(sizeof(double) * n_w);
    HIPC(hipMemcpyAsync(wd.p, w_grid, sizeof(double) * n_w, hipMemcpyHostToDevice, st));
  }
  double* buf = fv.as<double>();
  auto vec = [&](int p, int k) { return buf + ((size_t)p * 3 + (size_t)(k % 3)) * len; };
  const double* phv = s->phi64.as<double>() + (size_t)(S - n_o) * ng;
  for (int p = 0; p < 3; ++p) {
    double* f0 = vec(p, 0);
    HIPC(launch_mixed_dipole(phv, n_o, s->n, s->cfg.h, p, f0, st));
    proj_coef(f0, n_o, s->phi64.as<double>(), S, ng, s->dv, pq.as<double>(), cq.as<double>(), st);
    HIPC(launch_project_out(f0, n_o, s->phi64.as<double>(), S, cq.as<double>(), ng, st));
  }
  for (int k = 0; k < K; ++k)
    for (int p = 0; p < 3; ++p) {
      const double* fc = vec(p, k);
      apply_a_mixed_device(s, fc, af.as<double>());
      HIPC(launch_mixed_cheb_update(af.as<double>(), fc, vec(p, k + 2), vec(p, k + 1), len, a, b,
                                    k == 0 ? 1 : 0, s->dv, p, part.as<double>() + (size_t)k * nblk * 6,
                                    st));
    }
  HIPC(launch_cheb_spectrum(part.as<double>(), K, nblk, mu.as<double>(), M, D.as<double>(), a, b,
                            wd.as<double>(), n_w, sig, sd.as<double>(), st));
  if (n_w > 0) HIPC(hipMemcpyAsync(sigma, sd.p, sizeof(double) * n_w, hipMemcpyDeviceToHost, st));
  if (residues)
    HIPC(hipMemcpyAsync(residues, mu.p, sizeof(double) * 3 * (size_t)n_mom, hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
}

// The Chebyshev interval: the caller's [e_min, e_max] if e_min < e_max,
// otherwise the Gershgorin interval of the device copy of A
void cheb_interval(bse_system* s, int n, double* e_min, double* e_max, const char* who) {
  if (*e_min < *e_max) return;
  hipStream_t st = s->stream;
  DBuf lohi;
  lohi.alloc(sizeof(double) * 2 * (size_t)n);
  HIPC(launch_gershgorin(s->A_d.as<double>(), n, lohi.as<double>(), st));
  std::vector<double> h(2 * (size_t)n);
  HIPC(hipMemcpyAsync(h.data(), lohi.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  *e_min = *std::min_element(h.begin(), h.begin() + n);
  *e_max = *std::max_element(h.begin() + n, h.end());
  if (!(*e_min < *e_max)) fail(BSE_ERR_ARG, std::string(who) + ": degenerate interval; pass bounds");
}

// electron-hole dipoles of the last bse_build_A as three start vectors
// [3][n] on the device (f0_d holds them as [n][3])
void cheb_start(bse_system* s, int n, double* dst) {
  hipStream_t st = s->stream;
  std::vector<double> f0(3 * (size_t)n), f0t(3 * (size_t)n);
  HIPC(hipMemcpyAsync(f0.data(), s->f0_d.p, sizeof(double) * f0.size(), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  for (int i = 0; i < n; ++i)
    for (int p = 0; p < 3; ++p) f0t[(size_t)p * n + i] = f0[(size_t)i * 3 + p];
  HIPC(hipMemcpyAsync(dst, f0t.data(), sizeof(double) * f0t.size(), hipMemcpyHostToDevice, st));
  HIPC(hipStreamSynchronize(st));
}

// Chebyshev absorption (Eqs. 7-8) on the device copy of A: the residues of
// the three dipole start vectors by the recursion in A~ = (A - b)/a, then the
// broadened delta through its Chebyshev coefficients (Gauss-Chebyshev
// quadrature on M = 2 n_mom nodes, summed at the nodes).
void chebyshev_spectrum(bse_system* s, int n_mom, double e_min, double e_max, int n_w,
                        const double* w_grid, double sig, double* sigma, double* residues,
                        double* bounds) {
  if (!s) fail(BSE_ERR_ARG, "null system");
  if (s->a_no == 0) fail(BSE_ERR_STATE, "bse_chebyshev_spectrum: call bse_build_A first");
  const int n = s->a_no * s->a_nc;
  if (n_mom < 2 || n_mom % 2 != 0 || n_w < 0 || (n_w > 0 && (!w_grid || !sigma || !(sig > 0))) ||
      (n_w == 0 && !residues))
    fail(BSE_ERR_ARG, "bse_chebyshev_spectrum: bad arguments");
  hipStream_t st = s->stream;
  const double* A = s->A_d.as<double>();
  cheb_interval(s, n, &e_min, &e_max, "bse_chebyshev_spectrum");
  const double b = 0.5 * (e_max + e_min), a = 0.5 * (e_max - e_min) * 1.01;
  const int K = n_mom / 2, nblk = cheb_blocks(n), M = 2 * n_mom;
  DBuf fv, part, mu, D, wd, sd;
  fv.alloc(sizeof(double) * 9 * (size_t)n);
  part.alloc(sizeof(double) * 6 * (size_t)K * nblk);
  mu.alloc(sizeof(double) * 3 * (size_t)n_mom);
  D.alloc(sizeof(double) * 3 * (size_t)M);
  if (n_w > 0) {
    wd.alloc(sizeof(double) * n_w);
    sd.alloc(sizeof(double) * n_w);
    HIPC(hipMemcpyAsync(wd.p, w_grid, sizeof(double) * n_w, hipMemcpyHostToDevice, st));
  }
  // f^0 = dipoles, [3][n]
  double* buf = fv.as<double>();
  cheb_start(s, n, buf);
  for (int k = 0; k < K; ++k) {
    const double* fc = buf + (size_t)(k % 3) * 3 * n;
    const double* fp = buf + (size_t)((k + 2) % 3) * 3 * n;
    double* fn = buf + (size_t)((k + 1) % 3) * 3 * n;
    HIPC(launch_cheb_step(A, n, fc, fp, fn, a, b, k == 0 ? 1 : 0,
                          part.as<double>() + (size_t)k * nblk * 6, st));
  }
  HIPC(launch_cheb_spectrum(part.as<double>(), K, nblk, mu.as<double>(), M, D.as<double>(), a, b,
                            wd.as<double>(), n_w, sig, sd.as<double>(), st));
  if (n_w > 0) HIPC(hipMemcpyAsync(sigma, sd.p, sizeof(double) * n_w, hipMemcpyDeviceToHost, st));
  if (residues)
    HIPC(hipMemcpyAsync(residues, mu.p, sizeof(double) * 3 * (size_t)n_mom, hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  if (bounds) {
    bounds[0] = e_min;
    bounds[1] = e_max;
  }
}

// chebyshev_spectrum without allocation: the same launches and arithmetic,
// with every device buffer carved from this device's `scratch` array and no
// host staging (start vectors and the Gershgorin interval on the device).
// Sizes in doubles, each part rounded up to 256 bytes.
size_t cheb_noalloc_doubles(int n, int n_mom, int n_w) {
  auto r = [](size_t x) { return (x + 31) / 32 * 32; };
  const size_t K = (size_t)n_mom / 2, nblk = (size_t)cheb_blocks(n), M = 2 * (size_t)n_mom;
  return r(9 * (size_t)n) + r(6 * K * nblk) + r(3 * (size_t)n_mom) + r(3 * M) + 2 * r((size_t)n_w) +
         r(2 * (size_t)n) + r(2);
}

void chebyshev_spectrum_noalloc(bse_system* s, int n_mom, double e_min, double e_max, int n_w,
                                const double* w_grid, double sig, double* sigma, double* residues,
                                double* bounds) {
  if (!s) fail(BSE_ERR_ARG, "null system");
  if (s->a_no == 0) fail(BSE_ERR_STATE, "bse_chebyshev_spectrum_noalloc: call bse_build_A first");
  const int n = s->a_no * s->a_nc;
  if (n_mom < 2 || n_mom % 2 != 0 || n_w < 0 || (n_w > 0 && (!w_grid || !sigma || !(sig > 0))) ||
      (n_w == 0 && !residues))
    fail(BSE_ERR_ARG, "bse_chebyshev_spectrum_noalloc: bad arguments");
  if (cheb_noalloc_doubles(n, n_mom, n_w) * sizeof(double) > NOALLOC_SCRATCH_BYTES)
    fail(BSE_ERR_ARG, "bse_chebyshev_spectrum_noalloc: n_mom, n_w and the size of A need more than the "
                      "64 MiB of scratch (about 0.75 n_mom n_ia + 9 n_ia + 9 n_mom + 2 n_w doubles)");
  double* base = scratch_dev(s->cfg.device);
  if (!base) fail(BSE_ERR_STATE, "bse_chebyshev_spectrum_noalloc: no scratch on this device");
  HIPC(hipSetDevice(s->cfg.device));
  hipStream_t st = s->stream;
  auto r = [](size_t x) { return (x + 31) / 32 * 32; };
  const int K = n_mom / 2, nblk = cheb_blocks(n), M = 2 * n_mom;
  double* fv = base;
  double* part = fv + r(9 * (size_t)n);
  double* mu = part + r(6 * (size_t)K * nblk);
  double* D = mu + r(3 * (size_t)n_mom);
  double* wd = D + r(3 * (size_t)M);
  double* sd = wd + r((size_t)n_w);
  double* lohi = sd + r((size_t)n_w);
  double* mm = lohi + r(2 * (size_t)n);
  const double* A = s->A_d.as<double>();
  if (!(e_min < e_max)) {
    double h[2];
    HIPC(launch_gershgorin(A, n, lohi, st));
    HIPC(launch_interval(lohi, n, mm, st));
    HIPC(hipMemcpyAsync(h, mm, sizeof(h), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    e_min = h[0];
    e_max = h[1];
    if (!(e_min < e_max)) fail(BSE_ERR_ARG, "bse_chebyshev_spectrum_noalloc: degenerate interval; pass bounds");
  }
  const double b = 0.5 * (e_max + e_min), a = 0.5 * (e_max - e_min) * 1.01;
  if (n_w > 0) HIPC(hipMemcpyAsync(wd, w_grid, sizeof(double) * n_w, hipMemcpyHostToDevice, st));
  HIPC(launch_cheb_start(s->f0_d.as<double>(), n, fv, st));
  for (int k = 0; k < K; ++k) {
    const double* fc = fv + (size_t)(k % 3) * 3 * n;
    const double* fp = fv + (size_t)((k + 2) % 3) * 3 * n;
    double* fn = fv + (size_t)((k + 1) % 3) * 3 * n;
    HIPC(launch_cheb_step(A, n, fc, fp, fn, a, b, k == 0 ? 1 : 0, part + (size_t)k * nblk * 6, st));
  }
  HIPC(launch_cheb_spectrum(part, K, nblk, mu, M, D, a, b, wd, n_w, sig, sd, st));
  if (n_w > 0) HIPC(hipMemcpyAsync(sigma, sd, sizeof(double) * n_w, hipMemcpyDeviceToHost, st));
  if (residues) HIPC(hipMemcpyAsync(residues, mu, sizeof(double) * 3 * (size_t)n_mom, hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  if (bounds) {
    bounds[0] = e_min;
    bounds[1] = e_max;
  }
}

// Frequency-resolved exciton states (Eq. 8) on the device copy of A: the full
// three-term recursion from the dipole start vectors with
// F_q += g_m(omega_q) f^m at every step, then (optionally) the exciton
// densities 2 sum_ia F_ia phi_i phi_a of every (omega, polarisation).
void exciton_states(bse_system* s, int n_mom, double e_min, double e_max, int n_w, const double* w_list,
                    double sig, double* f_out, double* dens_out, double* bounds) {
  if (!s) fail(BSE_ERR_ARG, "null system");
  if (s->a_no == 0) fail(BSE_ERR_STATE, "bse_exciton_states: call bse_build_A first");
  if (n_mom < 2 || n_w < 1 || n_w > 8 || !w_list || !f_out || !(sig > 0))
    fail(BSE_ERR_ARG, "bse_exciton_states: bad arguments");
  const int n = s->a_no * s->a_nc;
  hipStream_t st = s->stream;
  const double* A = s->A_d.as<double>();
  cheb_interval(s, n, &e_min, &e_max, "bse_exciton_states");
  const double b = 0.5 * (e_max + e_min), a = 0.5 * (e_max - e_min) * 1.01;
  auto* t = s->timer.begin("exciton_states");
  DBuf fv, g, F, wd;
  fv.alloc(sizeof(double) * 9 * (size_t)n);
  g.alloc(sizeof(double) * (size_t)n_w * n_mom);
  F.alloc(sizeof(double) * 3 * (size_t)n_w * n);
  wd.alloc(sizeof(double) * n_w);
  HIPC(hipMemcpyAsync(wd.p, w_list, sizeof(double) * n_w, hipMemcpyHostToDevice, st));
  HIPC(launch_cheb_coef(wd.as<double>(), n_w, n_mom, 2 * n_mom, a, b, sig, g.as<double>(), st));
  double* buf = fv.as<double>();
  cheb_start(s, n, buf);
  HIPC(launch_cheb_acc_init(buf, n, g.as<double>(), n_mom, n_w, F.as<double>(), st));
  // buffer k % 3 holds f^k
  for (int m = 0; m + 1 < n_mom; ++m) {
    const double* fc = buf + (size_t)(m % 3) * 3 * n;
    const double* fp = buf + (size_t)((m + 2) % 3) * 3 * n;
    double* fn = buf + (size_t)((m + 1) % 3) * 3 * n;
    HIPC(launch_cheb_step_acc(A, n, fc, fp, fn, a, b, m == 0 ? 1 : 0, g.as<double>(), n_mom, m + 1, n_w,
                              F.as<double>(), st));
  }
  const size_t ng = s->ng;
  DBuf dens;
  if (dens_out) {
    const int v0 = s->cfg.n_occ - s->a_no, c0 = s->cfg.n_occ;
    dens.alloc(sizeof(double) * 3 * (size_t)n_w * ng);
    HIPC(launch_exciton_density(s->phi64.as<double>(), v0, c0, s->a_no, s->a_nc, ng, F.as<double>(),
                                3 * n_w, dens.as<double>(), st));
  }
  s->timer.end(t);
  HIPC(hipMemcpyAsync(f_out, F.p, sizeof(double) * 3 * (size_t)n_w * n, hipMemcpyDeviceToHost, st));
  if (dens_out)
    HIPC(hipMemcpyAsync(dens_out, dens.p, sizeof(double) * 3 * (size_t)n_w * ng, hipMemcpyDeviceToHost,
                        st));
  HIPC(hipStreamSynchronize(st));
  if (bounds) {
    bounds[0] = e_min;
    bounds[1] = e_max;
  }
}

// Frequency-resolved exciton states of the mixed representation (Eq. 8 with
// the matrix-free A of Eq. 6), one polarisation at a time: the full
// recursion on the grid vectors f_j(r) from the mixed dipole start with
// F_q += g_m(omega_q) f^m at every step, then the electron-hole amplitudes
// f_ia = h^3 sum_r phi_a f_i on the n_a lowest virtual orbitals and the
// exciton densities 2 sum_i phi_i f_i.
void exciton_states_mixed(bse_system* s, int n_mom, double e_min, double e_max, int n_w,
                          const double* w_list, double sig, int n_a, double* f_out, double* dens_out) {
  if (!s) fail(BSE_ERR_ARG, "null system");
  if (s->a_no == 0) fail(BSE_ERR_STATE, "bse_exciton_states_mixed: call bse_build_A first");
  const int n_o = s->a_no, S = s->cfg.n_occ;
  const int n_virt = s->n_orb - S;
  if (n_mom < 2 || !(e_min < e_max) || n_w < 1 || n_w > 8 || !w_list || !(sig > 0) || n_a < 0 ||
      n_a > n_virt || (n_a > 0 && !f_out) || (n_a == 0 && !dens_out))
    fail(BSE_ERR_ARG, "bse_exciton_states_mixed: bad arguments");
  if ((size_t)n_o * S * sizeof(double) > 64 * 1024)
    fail(BSE_ERR_ARG, "bse_exciton_states_mixed: n_o * n_occ above 8192");
  hipStream_t st = s->stream;
  const size_t ng = s->ng, len = (size_t)n_o * ng;
  const double b = 0.5 * (e_max + e_min), a = 0.5 * (e_max - e_min) * 1.01;
  DBuf fv, af, part, g, F, wd, cq, pq, amp, pa, rho;
  fv.alloc(sizeof(double) * 3 * len);               // [3 rotating vectors][n_o][ng]
  af.alloc(sizeof(double) * len);
  part.alloc(sizeof(double) * 6 * (size_t)mixed_cheb_blocks());
  g.alloc(sizeof(double) * (size_t)n_w * n_mom);
  F.alloc(sizeof(double) * (size_t)n_w * len);
  wd.alloc(sizeof(double) * n_w);
  cq.alloc(sizeof(double) * (size_t)n_o * S);
  pq.alloc(sizeof(double) * std::max(proj_scratch(n_o, S, ng), proj_scratch(n_o, std::max(n_a, 1), ng)));
  if (n_a > 0) amp.alloc(sizeof(double) * (size_t)n_o * n_a);
  if (dens_out) rho.alloc(sizeof(double) * ng);
  HIPC(hipMemcpyAsync(wd.p, w_list, sizeof(double) * n_w, hipMemcpyHostToDevice, st));
  HIPC(launch_cheb_coef(wd.as<double>(), n_w, n_mom, 2 * n_mom, a, b, sig, g.as<double>(), st));
  double* buf = fv.as<double>();
  auto vec = [&](int k) { return buf + (size_t)(k % 3) * len; };
  const double* phv = s->phi64.as<double>() + (size_t)(S - n_o) * ng;
  const double* pha = s->phi64.as<double>() + (size_t)S * ng;
  auto* t = s->timer.begin("exciton_states_mixed");
  for (int p = 0; p < 3; ++p) {
    double* f0 = vec(0);
    HIPC(launch_mixed_dipole(phv, n_o, s->n, s->cfg.h, p, f0, st));
    proj_coef(f0, n_o, s->phi64.as<double>(), S, ng, s->dv, pq.as<double>(), cq.as<double>(), st);
    HIPC(launch_project_out(f0, n_o, s->phi64.as<double>(), S, cq.as<double>(), ng, st));
    HIPC(launch_states_acc(F.as<double>(), f0, g.as<double>(), n_mom, 0, n_w, len, 1, st));
    for (int m = 0; m + 1 < n_mom; ++m) {
      apply_a_mixed_device(s, vec(m), af.as<double>());
      HIPC(launch_mixed_cheb_update(af.as<double>(), vec(m), vec(m + 2), vec(m + 1), len, a, b,
                                    m == 0 ? 1 : 0, s->dv, p, part.as<double>(), st));
      HIPC(launch_states_acc(F.as<double>(), vec(m + 1), g.as<double>(), n_mom, m + 1, n_w, len, 0, st));
    }
    for (int q = 0; q < n_w; ++q) {
      const double* Fq = F.as<double>() + (size_t)q * len;
      if (n_a > 0) {
        proj_coef(Fq, n_o, pha, n_a, ng, s->dv, pq.as<double>(), amp.as<double>(), st);
        HIPC(hipMemcpyAsync(f_out + ((size_t)q * 3 + p) * n_o * n_a, amp.p, sizeof(double) * n_o * n_a,
                            hipMemcpyDeviceToHost, st));
      }
      if (dens_out) {
        HIPC(launch_mixed_density(phv, Fq, n_o, ng, rho.as<double>(), st));
        HIPC(hipMemcpyAsync(dens_out + ((size_t)q * 3 + p) * ng, rho.p, sizeof(double) * ng,
                            hipMemcpyDeviceToHost, st));
      }
      HIPC(hipStreamSynchronize(st));   // amp and rho are reused
    }
  }
  s->timer.end(t);
  HIPC(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------------------
// autotuner: x-tile width and plane-pass block size for this system's grid,
// batch size and precision, timed on the system's own buffers; results are
// appended to a text cache (one "key tc nt ms_x ms_yz" line per shape)
// ---------------------------------------------------------------------------
template <typename T>
float time_launches(bse_system* s, int reps, const std::function<hipError_t()>& fn) {
  hipEvent_t a, b;
  HIPC(hipEventCreate(&a));
  HIPC(hipEventCreate(&b));
  hipError_t e = fn();  // warm-up, also validates the variant
  if (e != hipSuccess) {
    (void)hipGetLastError();
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return -1.f;
  }
  HIPC(hipEventRecord(a, s->stream));
  for (int r = 0; r < reps; ++r) HIPC(fn());
  HIPC(hipEventRecord(b, s->stream));
  HIPC(hipEventSynchronize(b));
  float ms = 0;
  HIPC(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms / reps;
}

template <typename T>
void autotune_t(bse_system* s, int B, const char* cache_path) {
  using C = cplx<T>;
  char key[128];
  std::snprintf(key, sizeof(key), "n%d_%s_B%d_L%d", s->n, sizeof(T) == 4 ? "f32" : "f64", B, s->L);
  // the choices a result sets: the x tile, the plane block size (0 where
  // the y-z factors run as one register-line pass), the x pass's workgroup
  // order, and for the one-pass y-z kernel its 16-point DFT schedule and order
  auto apply = [&](int tc, int nt, int ox, int sched, int oz) {
    s->tune_tc = tc;
    s->tune_nt = nt;
    s->launch_order = (s->launch_order & ~1) | (ox & 1);
    // a schedule is kept only where the one-pass y-z kernel runs (not after
    // bse_set_yz_schedule chose the line passes)
    if (sched >= 0 && s->yz_schedule != 1 && prop_yz_fused<T>(s->n)) {
      s->yz_schedule = sched;
      s->launch_order = (s->launch_order & ~4) | ((oz & 1) << 2);
    }
  };
  if (cache_path && *cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream is(line);
      std::string k;
      int tc = 0, nt = 0, ox = s->launch_order & 1, sched = -1, oz = 0;
      float mx = 0, myz = 0;
      if (is >> k >> tc >> nt && k == key) {
        // lines written before the orders were tuned end after the times
        if (is >> mx >> myz >> ox) is >> sched >> oz;
        apply(tc, nt, ox, sched, oz);
        return;
      }
    }
  }
  ensure_batch<T>(s, B);
  Tables& tb = tabs<T>(s);
  HIPC(launch_fill_zero(s->d.p, sizeof(C) * s->ng * (size_t)B * s->L, s->stream));
  HIPC(launch_fill_zero(s->u.p, sizeof(T) * s->ng * (size_t)B, s->stream));
  PropXArgs<T> px = prop_pair_x_args<T>(s, s->h0.as<C>(), false);
  PropYZArgs<T> pz = prop_pair_yz_args<T>(s, s->h0.as<C>());
  float best_x = 1e30f, best_yz = 1e30f;
  int tc_best = 0, nt_best = 0, ox_best = 0, sched_best = -1, oz_best = 0;
  for (int ox : {0, 1})
    for (int tc : {16, 32, 64}) {
      px.order = ox;
      const float ms = time_launches<T>(s, 5, [&]() { return launch_prop_x<T>(s->n, px, B, s->stream, tc); });
      if (ms > 0 && ms < best_x) { best_x = ms; tc_best = tc; ox_best = ox; }
    }
  if (s->yz_schedule != 1 && prop_yz_fused<T>(s->n)) {
    for (int sched : {2, 0})
      for (int oz : {0, 1}) {
        pz.fused = sched == 2 ? 2 : 1;
        pz.order = oz;
        const float ms = time_launches<T>(s, 5, [&]() { return launch_prop_yz<T>(s->n, pz, B, s->stream, 0); });
        if (ms > 0 && ms < best_yz) { best_yz = ms; sched_best = sched; oz_best = oz; }
      }
    if (sched_best < 0) fail(BSE_ERR_DEVICE, "autotune: no valid variant");
  } else {
    for (int nt : {256, 512}) {
      const float ms = time_launches<T>(s, 5, [&]() { return launch_prop_yz<T>(s->n, pz, B, s->stream, nt); });
      if (ms > 0 && ms < best_yz) { best_yz = ms; nt_best = nt; }
    }
    if (nt_best == 0) fail(BSE_ERR_DEVICE, "autotune: no valid variant");
  }
  if (tc_best == 0) fail(BSE_ERR_DEVICE, "autotune: no valid variant");
  apply(tc_best, nt_best, ox_best, sched_best, oz_best);
  if (cache_path && *cache_path) {
    std::ofstream out(cache_path, std::ios::app);
    out << key << " " << tc_best << " " << nt_best << " " << best_x << " " << best_yz << " " << ox_best << " "
        << sched_best << " " << oz_best << "\n";
  }
}

// ---------------------------------------------------------------------------
// lockstep work-list schedule of an uneven batch: every system takes time
// step n in turn, and the perturbed sets' x and plane passes of all systems
// of one grid size run as one persistent work-list launch each, over the
// (system, pair, tile or plane) items of those systems.  The pass arguments of a step depend
// only on which buffer holds H_n (h0 at n = 0, then hbuf[n & 1]), on whether
// the state is an end-of-step one (t = 0 or just cleaned) and on which
// buffer takes H_{n+1}, so every variant is on the device before the first
// step and the schedule can be captured.
// ---------------------------------------------------------------------------
void batch_list_check(int n_sys, bse_system* const* sys) {
  for (int i = 0; i < n_sys; ++i) {
    const bse_system* s = sys[i];
    if (s->cfg.precision != BSE_MIXED)
      fail(BSE_ERR_ARG, "bse_apply_W_batch: the work-list schedule runs mixed-precision systems only");
    if (!prop_list_grid(s->n) || prop_yz_split<float>(s->n) || prop_yz_fused<float>(s->n))
      fail(BSE_ERR_ARG, "bse_apply_W_batch: the work-list schedule takes grids of 16, 24, 32, 48 or 64 points per axis");
    if (s->cfg.n_steps != sys[0]->cfg.n_steps || s->cfg.clean_every != sys[0]->cfg.clean_every)
      fail(BSE_ERR_ARG, "bse_apply_W_batch: the work-list schedule needs the same number of steps and cleaning "
                        "interval in every system");
  }
}

constexpr int LIST_XV = 5;   // x-pass variants: n = 0, then (n & 1, end-of-step state)

// the systems grouped by grid size; in each group's entries, first counts
// the group's items before the system
struct BatchList {
  struct Group {
    int n;
    int e0, ne;              // entries e0 .. e0 + ne - 1 of every variant
    unsigned tot_x, tot_yz;
  };
  std::vector<Group> groups;
  DBuf buf;                  // LIST_XV x n_sys XListSys, then 2 x n_sys YZListSys
  int n_sys = 0;
  const XListSys* x(int v, const Group& g) const { return buf.as<XListSys>() + (size_t)v * n_sys + g.e0; }
  const YZListSys* yz(int p, const Group& g) const {
    return reinterpret_cast<const YZListSys*>(buf.as<XListSys>() + (size_t)LIST_XV * n_sys) + (size_t)p * n_sys +
           g.e0;
  }
};

void batch_list_build(int n_sys, bse_system* const* sys, const int32_t* n_pairs, BatchList& bl) {
  std::vector<XListSys> xl((size_t)LIST_XV * n_sys);
  std::vector<YZListSys> yl((size_t)2 * n_sys);
  bl.n_sys = n_sys;
  std::vector<int> order(n_sys);
  for (int i = 0; i < n_sys; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int p, int q) { return sys[p]->n < sys[q]->n; });
  for (int k = 0; k < n_sys; ++k) {
    const int i = order[k];
    bse_system* s = sys[i];
    const int B = n_pairs[i];
    if (bl.groups.empty() || bl.groups.back().n != s->n) bl.groups.push_back({s->n, k, 0, 0u, 0u});
    BatchList::Group& g = bl.groups.back();
    for (int v = 0; v < LIST_XV; ++v) {
      const cplx<float>* hcur = v == 0 ? s->h0.as<cplx<float>>() : prop_hbuf<float>(s, (v - 1) >> 1);
      const bool half = v == 0 || ((v - 1) & 1);
      XListSys& e = xl[(size_t)v * n_sys + k];
      e.a = prop_pair_x_args<float>(s, hcur, half);
      e.a.nf = B;
      e.first = g.tot_x;
    }
    for (int p = 0; p < 2; ++p) {
      YZListSys& e = yl[(size_t)p * n_sys + k];
      e.a = prop_pair_yz_args<float>(s, prop_hbuf<float>(s, p));
      e.a.nf = B;
      e.first = g.tot_yz;
    }
    g.ne += 1;
    g.tot_x += prop_x_list_items(s->n, B);
    g.tot_yz += prop_yz_list_items(s->n, B);
  }
  const size_t bx = sizeof(XListSys) * xl.size(), by = sizeof(YZListSys) * yl.size();
  bl.buf.alloc(bx + by);
  HIPC(hipMemcpy(bl.buf.p, xl.data(), bx, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(static_cast<char*>(bl.buf.p) + bx, yl.data(), by, hipMemcpyHostToDevice));
}

// the whole batch on one stream (every system's stream set to it)
void batch_list_run(int n_sys, bse_system* const* sys, const int32_t* n_pairs, void* const* w_dev,
                    const BatchList& bl, hipStream_t st) {
  std::vector<PropRun<float>> runs(n_sys);
  for (int i = 0; i < n_sys; ++i) {
    runs[i] = PropRun<float>{sys[i], n_pairs[i], sys[i]->pq_d.as<int>(), nullptr, true};
    prop_begin<float>(runs[i]);
  }
  const int N = sys[0]->cfg.n_steps;
  for (int n = 0; n < N; ++n) {
    for (auto& r : runs) prop_unperturbed_step<float>(r, n, r.s->stream);
    const int v = n == 0 ? 0 : 1 + 2 * (n & 1) + (runs[0].half ? 1 : 0);
    for (const auto& g : bl.groups) HIPC(launch_prop_x_list(g.n, bl.x(v, g), g.ne, g.tot_x, st));
    for (const auto& g : bl.groups) HIPC(launch_prop_yz_list(g.n, bl.yz((n + 1) & 1, g), g.ne, g.tot_yz, st));
    for (auto& r : runs) prop_after_passes<float>(r, n);
  }
  for (int i = 0; i < n_sys; ++i) {
    bse_system* s = sys[i];
    double* w = reinterpret_cast<double*>(w_dev[i]);
    HIPC(launch_add(s->q.as<double>(), s->wpol.as<double>(), (size_t)n_pairs[i] * s->ng, w, st));
    HIPC(launch_finite_check(w, n_pairs[i], s->ng, s->flags.as<int>(), st));
    HIPC(launch_nan_flagged(w, n_pairs[i], s->ng, s->flags.as<int>(), st));
  }
}

// ---------------------------------------------------------------------------
// uneven batch: several systems (grids, pair counts) propagated together.
// mode bit 0: the whole propagation captured into one HIP graph and launched
// once; bit 1: the lockstep work-list schedule on one stream, else every
// system on its own stream (one graph branch each when captured)
// ---------------------------------------------------------------------------
void apply_w_batch(int n_sys, bse_system* const* sys, const int32_t* n_pairs,
                   const int32_t* const* pq, void* const* w_dev, int mode) {
  if (n_sys < 1 || !sys || !n_pairs || !pq || !w_dev) fail(BSE_ERR_ARG, "bse_apply_W_batch: null argument");
  if (mode < 0 || mode > 3) fail(BSE_ERR_ARG, "bse_apply_W_batch: mode must be 0..3");
  const bool use_graph = (mode & 1) != 0, list = (mode & 2) != 0;
  int dev = -1;
  for (int i = 0; i < n_sys; ++i) {
    bse_system* s = sys[i];
    check_ready(s);
    if (dev < 0) dev = s->cfg.device;
    if (s->cfg.device != dev) fail(BSE_ERR_ARG, "bse_apply_W_batch: systems on different devices");
    if (n_pairs[i] < 1 || n_pairs[i] > s->cfg.max_batch || !pq[i] || !w_dev[i])
      fail(BSE_ERR_ARG, "bse_apply_W_batch: need 1 <= n_pairs <= max_batch and non-null buffers");
    for (int j = i + 1; j < n_sys; ++j)
      if (sys[j] == s) fail(BSE_ERR_ARG, "bse_apply_W_batch: a system appears twice");
    for (int k = 0; k < n_pairs[i]; ++k)
      if (pq[i][2 * k] < 0 || pq[i][2 * k] >= s->n_orb || pq[i][2 * k + 1] < 0 || pq[i][2 * k + 1] >= s->n_orb)
        fail(BSE_ERR_ARG, "pair index out of range");
  }
  if (list) batch_list_check(n_sys, sys);
  HIPC(hipSetDevice(dev));
  std::vector<hipStream_t> saved(n_sys);
  std::vector<char> timer_was(n_sys, 0);
  for (int i = 0; i < n_sys; ++i) {
    bse_system* s = sys[i];
    if (!s->own_stream) HIPC(hipStreamCreateWithFlags(&s->own_stream, hipStreamNonBlocking));
    saved[i] = s->stream;
    timer_was[i] = s->timer.on ? 1 : 0;
  }
  hipStream_t origin = nullptr;
  std::vector<hipEvent_t> ev(n_sys + 1, nullptr), pre(n_sys, nullptr);
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto restore = [&]() {
    for (int i = 0; i < n_sys; ++i) {
      sys[i]->stream = saved[i];
      sys[i]->timer.on = timer_was[i] != 0;
    }
    for (auto e : ev) if (e) (void)hipEventDestroy(e);
    for (auto e : pre) if (e) (void)hipEventDestroy(e);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (origin) (void)hipStreamDestroy(origin);
  };
  try {
    HIPC(hipStreamCreateWithFlags(&origin, hipStreamNonBlocking));
    for (auto& e : ev) HIPC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto& e : pre) HIPC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    // the batch reuses each system's workspace and writes the caller's
    // buffers: it starts after the work already queued on every system's
    // stream (a device W-action still running, the caller's fill of w_dev)
    for (int i = 0; i < n_sys; ++i) {
      bse_system* s = sys[i];
      HIPC(hipEventRecord(pre[i], saved[i]));
      HIPC(hipStreamWaitEvent(origin, pre[i], 0));
      HIPC(hipStreamWaitEvent(s->own_stream, pre[i], 0));
      if (s->cfg.precision == BSE_FP64) ensure_batch<double>(s, n_pairs[i]);
      else ensure_batch<float>(s, n_pairs[i]);
      HIPC(hipMemcpyAsync(s->pq_d.p, pq[i], sizeof(int) * 2 * n_pairs[i], hipMemcpyHostToDevice, s->own_stream));
      s->stream = list ? origin : s->own_stream;
      s->timer.on = false;
    }
    // the pair lists are on the device before the captured work reads them
    for (int i = 0; i < n_sys; ++i) HIPC(hipStreamSynchronize(sys[i]->own_stream));
    BatchList bl;
    if (list) batch_list_build(n_sys, sys, n_pairs, bl);
    if (use_graph) HIPC(hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal));
    HIPC(hipEventRecord(ev[n_sys], origin));
    if (list) batch_list_run(n_sys, sys, n_pairs, w_dev, bl, origin);
    for (int i = 0; i < n_sys && !list; ++i) {
      bse_system* s = sys[i];
      HIPC(hipStreamWaitEvent(s->stream, ev[n_sys], 0));
      const int B = n_pairs[i];
      if (s->cfg.precision == BSE_FP64) propagate_batch<double>(s, B, s->pq_d.as<int>());
      else propagate_batch<float>(s, B, s->pq_d.as<int>());
      double* w = reinterpret_cast<double*>(w_dev[i]);
      HIPC(launch_add(s->q.as<double>(), s->wpol.as<double>(), (size_t)B * s->ng, w, s->stream));
      HIPC(launch_finite_check(w, B, s->ng, s->flags.as<int>(), s->stream));
      HIPC(launch_nan_flagged(w, B, s->ng, s->flags.as<int>(), s->stream));
      HIPC(hipEventRecord(ev[i], s->stream));
      HIPC(hipStreamWaitEvent(origin, ev[i], 0));
    }
    if (use_graph) {
      HIPC(hipStreamEndCapture(origin, &graph));
      HIPC(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      HIPC(hipGraphLaunch(exec, origin));
    }
    HIPC(hipStreamSynchronize(origin));
  } catch (...) {
    if (use_graph) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(origin, &g);
      if (g) (void)hipGraphDestroy(g);
    }
    restore();
    throw;
  }
  restore();
}

// ---------------------------------------------------------------------------
// batch plan: the whole propagation of an uneven batch captured into one
// HIP graph once, replayed by every run (capture and instantiation stay out
// of the runs); each system on its own branch, pair lists in the plan's own
// device buffers
// ---------------------------------------------------------------------------
// the device addresses the captured kernels use: a run is refused when any
// of them has changed since the capture (a workspace grown by a larger
// batch, new orbitals of another size)
std::vector<const void*> workspace_signature(const bse_system* s) {
  const DBuf* bufs[] = {&s->d, &s->u, &s->dens, &s->wpol, &s->q, &s->rho64, &s->work, &s->work64,
                        &s->part, &s->part32, &s->gpart, &s->coef, &s->coefE, &s->E, &s->flags,
                        &s->pscale, &s->normpart, &s->phi64, &s->phi_occ32, &s->phih, &s->phil,
                        &s->phith, &s->phitl, &s->eta0, &s->h0, &s->hbuf, &s->n0,
                        &s->tf.tw, &s->tf.kph, &s->tf.pf, &s->tf.ph, &s->tf.k2,
                        &s->td.tw, &s->td.kph, &s->td.pf, &s->td.ph, &s->td.k2};
  std::vector<const void*> sig;
  for (const DBuf* b : bufs) sig.push_back(b->p);
  sig.push_back(reinterpret_cast<const void*>((uintptr_t)s->cap_b));
  return sig;
}

}  // namespace

struct bse_batch_plan {
  std::vector<bse_system*> sys;
  std::vector<int> npairs;
  std::vector<DBuf> pq;
  std::vector<std::vector<const void*>> sig;
  hipStream_t origin = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipEvent_t> pre;
  hipEvent_t done = nullptr;
  int device = 0;
  ~bse_batch_plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto e : pre) if (e) (void)hipEventDestroy(e);
    if (done) (void)hipEventDestroy(done);
    if (origin) (void)hipStreamDestroy(origin);
  }
};

namespace {

void plan_create(int n_sys, bse_system* const* sys, const int32_t* n_pairs, const int32_t* const* pq,
                 void* const* w_dev, bse_batch_plan** out) {
  if (n_sys < 1 || !sys || !n_pairs || !pq || !w_dev || !out) fail(BSE_ERR_ARG, "bse_batch_plan_create: null argument");
  int dev = -1;
  for (int i = 0; i < n_sys; ++i) {
    bse_system* s = sys[i];
    check_ready(s);
    if (dev < 0) dev = s->cfg.device;
    if (s->cfg.device != dev) fail(BSE_ERR_ARG, "bse_batch_plan_create: systems on different devices");
    if (n_pairs[i] < 1 || n_pairs[i] > s->cfg.max_batch || !pq[i] || !w_dev[i])
      fail(BSE_ERR_ARG, "bse_batch_plan_create: need 1 <= n_pairs <= max_batch and non-null buffers");
    for (int j = i + 1; j < n_sys; ++j)
      if (sys[j] == s) fail(BSE_ERR_ARG, "bse_batch_plan_create: a system appears twice");
    check_pairs(s, n_pairs[i], pq[i]);
  }
  HIPC(hipSetDevice(dev));
  auto* P = new bse_batch_plan();
  std::vector<hipStream_t> saved(n_sys);
  std::vector<char> timer_was(n_sys, 0);
  std::vector<hipEvent_t> ev(n_sys + 1, nullptr);
  auto restore = [&]() {
    for (int i = 0; i < n_sys; ++i) {
      sys[i]->stream = saved[i];
      sys[i]->timer.on = timer_was[i] != 0;
    }
    for (auto e : ev) if (e) (void)hipEventDestroy(e);
  };
  try {
    P->device = dev;
    P->sys.assign(sys, sys + n_sys);
    P->npairs.assign(n_pairs, n_pairs + n_sys);
    P->pq.resize(n_sys);
    P->pre.assign(n_sys, nullptr);
    HIPC(hipStreamCreateWithFlags(&P->origin, hipStreamNonBlocking));
    HIPC(hipEventCreateWithFlags(&P->done, hipEventDisableTiming));
    for (auto& e : P->pre) HIPC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto& e : ev) HIPC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (int i = 0; i < n_sys; ++i) {
      bse_system* s = sys[i];
      if (!s->own_stream) HIPC(hipStreamCreateWithFlags(&s->own_stream, hipStreamNonBlocking));
      saved[i] = s->stream;
      timer_was[i] = s->timer.on ? 1 : 0;
      // the workspace is sized before the capture and must not move after it
      HIPC(hipStreamSynchronize(s->stream));
      if (s->cfg.precision == BSE_FP64) ensure_batch<double>(s, n_pairs[i]);
      else ensure_batch<float>(s, n_pairs[i]);
      P->pq[i].alloc(sizeof(int) * 2 * n_pairs[i]);
      HIPC(hipMemcpy(P->pq[i].p, pq[i], sizeof(int) * 2 * n_pairs[i], hipMemcpyHostToDevice));
      s->stream = s->own_stream;
      s->timer.on = false;
    }
    HIPC(hipStreamBeginCapture(P->origin, hipStreamCaptureModeThreadLocal));
    HIPC(hipEventRecord(ev[n_sys], P->origin));
    for (int i = 0; i < n_sys; ++i) {
      bse_system* s = sys[i];
      HIPC(hipStreamWaitEvent(s->stream, ev[n_sys], 0));
      const int B = n_pairs[i];
      if (s->cfg.precision == BSE_FP64) propagate_batch<double>(s, B, P->pq[i].as<int>());
      else propagate_batch<float>(s, B, P->pq[i].as<int>());
      double* w = reinterpret_cast<double*>(w_dev[i]);
      HIPC(launch_add(s->q.as<double>(), s->wpol.as<double>(), (size_t)B * s->ng, w, s->stream));
      HIPC(launch_finite_check(w, B, s->ng, s->flags.as<int>(), s->stream));
      HIPC(launch_nan_flagged(w, B, s->ng, s->flags.as<int>(), s->stream));
      HIPC(hipEventRecord(ev[i], s->stream));
      HIPC(hipStreamWaitEvent(P->origin, ev[i], 0));
    }
    HIPC(hipStreamEndCapture(P->origin, &P->graph));
    HIPC(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
    for (int i = 0; i < n_sys; ++i) P->sig.push_back(workspace_signature(sys[i]));
  } catch (...) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (P->origin && hipStreamIsCapturing(P->origin, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(P->origin, &g);
      if (g) (void)hipGraphDestroy(g);
    }
    restore();
    delete P;
    throw;
  }
  restore();
  *out = P;
}

// stream-ordered: after the work already on every system's stream; every
// system's stream then waits for the whole batch
void plan_run(bse_batch_plan* P) {
  if (!P) fail(BSE_ERR_ARG, "bse_batch_plan_run: null plan");
  for (size_t i = 0; i < P->sys.size(); ++i)
    if (workspace_signature(P->sys[i]) != P->sig[i])
      fail(BSE_ERR_STATE, "bse_batch_plan_run: a system's workspace or orbitals moved since the plan was "
                          "made (larger batch or new orbitals); make a new plan");
  HIPC(hipSetDevice(P->device));
  for (size_t i = 0; i < P->sys.size(); ++i) {
    HIPC(hipEventRecord(P->pre[i], P->sys[i]->stream));
    HIPC(hipStreamWaitEvent(P->origin, P->pre[i], 0));
  }
  HIPC(hipGraphLaunch(P->exec, P->origin));
  HIPC(hipEventRecord(P->done, P->origin));
  for (bse_system* s : P->sys) HIPC(hipStreamWaitEvent(s->stream, P->done, 0));
}

// ---------------------------------------------------------------------------
// finite-box W(k->0) correction (Results section): boundary potential of one
// box on the device, and the inverse-dielectric fit over several boxes
// ---------------------------------------------------------------------------
double boundary_potential(bse_system* s) {
  check_ready(s);
  const size_t ng = s->ng;
  hipStream_t st = s->stream;
  if (!s->vdev.p || s->vdev.bytes < sizeof(double) * ng) {
    s->vdev.alloc(sizeof(double) * ng);
    HIPC(hipMemcpy(s->vdev.p, s->vext.data(), sizeof(double) * ng, hipMemcpyHostToDevice));
  }
  s->bnd_n.alloc(sizeof(double) * ng);
  s->bnd_v.alloc(sizeof(double) * ng);
  s->bnd_part.alloc(sizeof(double) * (boundary_part_elems(s->n) + 1));
  // n = 2 sum_{s < N_occ} phi_s^2, v_H = v[n] (k = 0 term removed)
  HIPC(launch_ground_density(s->phi64.as<double>(), s->cfg.n_occ, ng, s->bnd_n.as<double>(), st));
  poisson64(s, s->bnd_n.as<double>(), 1, s->bnd_v.as<double>(), nullptr, 0.0);
  double* part = s->bnd_part.as<double>();
  double* out = part + boundary_part_elems(s->n);
  HIPC(launch_boundary_average(s->vdev.as<double>(), s->bnd_v.as<double>(), s->n, part, out, st));
  double v = 0;
  HIPC(hipMemcpyAsync(&v, out, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  return v;
}

// ---------------------------------------------------------------------------
// surrogate samples and surrogate W-action
// ---------------------------------------------------------------------------
void surrogate_descriptors(bse_system* s) {
  if (s->n0_scale > 0) return;
  s->n0dens.alloc(sizeof(double) * s->ng);
  HIPC(launch_ground_density(s->phi64.as<double>(), s->cfg.n_occ, s->ng, s->n0dens.as<double>(), s->stream));
  std::vector<double> h(s->ng);
  HIPC(hipMemcpyAsync(h.data(), s->n0dens.p, sizeof(double) * s->ng, hipMemcpyDeviceToHost, s->stream));
  HIPC(hipStreamSynchronize(s->stream));
  double m0 = 0, mv = 0;
  for (size_t i = 0; i < s->ng; ++i) {
    m0 = std::max(m0, std::fabs(h[i]));
    mv = std::max(mv, std::fabs(s->vext[i]));
  }
  s->vdev.alloc(sizeof(double) * s->ng);
  HIPC(hipMemcpy(s->vdev.p, s->vext.data(), sizeof(double) * s->ng, hipMemcpyHostToDevice));
  s->n0_scale = m0 > 0 ? 1.0 / m0 : 1.0;
  s->v_scale = mv > 0 ? 1.0 / mv : 1.0;
}

// q for the B pairs in s->pq_d (into s->q, rho into s->rho64) and their RMS
// scales (device s->fscale, host copy returned)
std::vector<double> source_and_scale(bse_system* s, int B) {
  HIPC(launch_pair_density(s->phi64.as<double>(), s->pq_d.as<int>(), B, s->ng, s->rho64.as<double>(), s->stream));
  poisson64(s, s->rho64.as<double>(), B, s->q.as<double>(), nullptr, 0.0);
  s->fdots.alloc(sizeof(double) * 3 * B);
  HIPC(launch_row_dots(s->q.as<double>(), nullptr, nullptr, B, s->ng, s->fdots.as<double>(), s->stream));
  std::vector<double> dots(3 * (size_t)B), sc(B);
  HIPC(hipMemcpyAsync(dots.data(), s->fdots.p, sizeof(double) * 3 * B, hipMemcpyDeviceToHost, s->stream));
  HIPC(hipStreamSynchronize(s->stream));
  for (int b = 0; b < B; ++b) {
    sc[b] = std::sqrt(dots[3 * (size_t)b] / (double)s->ng);
    if (!(sc[b] > 0)) fail(BSE_ERR_NUMERIC, "pair density with zero source potential");
  }
  s->fscale.alloc(sizeof(double) * B);
  HIPC(hipMemcpyAsync(s->fscale.p, sc.data(), sizeof(double) * B, hipMemcpyHostToDevice, s->stream));
  return sc;
}

void make_samples(bse_system* s, int n_pairs, const int32_t* pq, float* x, float* t, double* scale_out) {
  check_ready(s);
  if (n_pairs < 1 || !pq || !x) fail(BSE_ERR_ARG, "bse_fno_make_samples: bad arguments");
  for (int k = 0; k < n_pairs; ++k)
    if (pq[2 * k] < 0 || pq[2 * k] >= s->n_orb || pq[2 * k + 1] < 0 || pq[2 * k + 1] >= s->n_orb)
      fail(BSE_ERR_ARG, "pair index out of range");
  surrogate_descriptors(s);
  const int Bmax = std::max(1, s->cfg.max_batch);
  for (int k0 = 0; k0 < n_pairs; k0 += Bmax) {
    const int B = std::min(Bmax, n_pairs - k0);
    if (s->cfg.precision == BSE_FP64) ensure_batch<double>(s, B);
    else ensure_batch<float>(s, B);
    HIPC(hipMemcpyAsync(s->pq_d.p, pq + 2 * k0, sizeof(int) * 2 * B, hipMemcpyHostToDevice, s->stream));
    if (t) {
      if (s->cfg.precision == BSE_FP64) propagate_batch<double>(s, B, s->pq_d.as<int>());
      else propagate_batch<float>(s, B, s->pq_d.as<int>());
    }
    source_and_scale(s, B);
    HIPC(launch_features(s->q.as<double>(), s->fscale.as<double>(), s->n0dens.as<double>(), s->n0_scale,
                         s->vdev.as<double>(), s->v_scale, B, s->ng, x + (size_t)k0 * 3 * s->ng, s->stream));
    if (t)
      HIPC(launch_targets(s->wpol.as<double>(), s->fscale.as<double>(), B, s->ng, t + (size_t)k0 * s->ng,
                          s->stream));
    if (scale_out)
      HIPC(hipMemcpyAsync(scale_out + k0, s->fscale.p, sizeof(double) * B, hipMemcpyDeviceToDevice, s->stream));
  }
  HIPC(hipStreamSynchronize(s->stream));
}

// Surrogate W-action with the propagation as the judge of its error:
// 1. W = q + s net(x) for every pair (device), with the sign check of the
//    screened energy <rho|W^pol rho> < 0 < <rho|W rho>;
// 2. n_judge pairs spread over the list are propagated, and the relative
//    L2 error of the network on each of them is measured on the device;
// 3. the other predictions are kept only if every judged error is finite
//    and at most tol (and their own sign check passes); every pair not kept
//    -- all of them when the judge rejects the network -- gets the
//    propagation's W, and the judged pairs keep their propagated W.
void apply_w_surrogate(bse_system* s, bse_fno* net, int n_pairs, const int32_t* pq, double* w_dev, double tol,
                       int n_judge, int32_t* accepted, double* judged_err) {
  check_ready(s);
  if (!net || n_pairs < 1 || !pq || !w_dev || n_judge < 0 || n_judge > n_pairs || !std::isfinite(tol))
    fail(BSE_ERR_ARG, "bse_apply_W_surrogate: bad arguments");
  check_pairs(s, n_pairs, pq);
  surrogate_descriptors(s);
  const size_t ng = s->ng;
  const int Bmax = std::max(1, std::min(s->cfg.max_batch, bse_fno_max_batch(net)));
  std::vector<int32_t> sign_ok(n_pairs, 0);
  HIPC(bse_fno_set_stream(net, s->stream) == BSE_OK ? hipSuccess : hipErrorInvalidValue);
  // 1. predictions
  for (int k0 = 0; k0 < n_pairs; k0 += Bmax) {
    const int B = std::min(Bmax, n_pairs - k0);
    if (s->cfg.precision == BSE_FP64) ensure_batch<double>(s, B);
    else ensure_batch<float>(s, B);
    s->fx.alloc(sizeof(float) * 3 * ng * B);
    s->fy.alloc(sizeof(float) * ng * B);
    s->fwpol.alloc(sizeof(double) * ng * B);
    HIPC(hipMemcpyAsync(s->pq_d.p, pq + 2 * k0, sizeof(int) * 2 * B, hipMemcpyHostToDevice, s->stream));
    source_and_scale(s, B);
    HIPC(launch_features(s->q.as<double>(), s->fscale.as<double>(), s->n0dens.as<double>(), s->n0_scale,
                         s->vdev.as<double>(), s->v_scale, B, ng, s->fx.as<float>(), s->stream));
    if (bse_fno_forward(net, B, s->fx.p, s->fy.p) != BSE_OK)
      fail(BSE_ERR_DEVICE, std::string("surrogate forward: ") + bse_fno_last_error());
    HIPC(launch_assemble_w(s->q.as<double>(), s->fscale.as<double>(), s->fy.as<float>(), B, ng,
                           s->fwpol.as<double>(), w_dev + (size_t)k0 * ng, s->stream));
    HIPC(launch_row_dots(s->rho64.as<double>(), s->q.as<double>(), s->fwpol.as<double>(), B, ng,
                         s->fdots.as<double>(), s->stream));
    std::vector<double> dots(3 * (size_t)B);
    HIPC(hipMemcpyAsync(dots.data(), s->fdots.p, sizeof(double) * 3 * B, hipMemcpyDeviceToHost, s->stream));
    HIPC(hipStreamSynchronize(s->stream));
    for (int b = 0; b < B; ++b) {
      const double e0 = dots[3 * (size_t)b + 1], e = dots[3 * (size_t)b + 2];
      sign_ok[k0 + b] = (std::isfinite(e) && e < 0.0 && e > -e0) ? 1 : 0;
    }
  }
  // 2. the judge: propagate a spread sample and measure the network's error
  std::vector<int> jidx(n_judge);
  std::vector<char> is_judged(n_pairs, 0);
  for (int k = 0; k < n_judge; ++k) {
    jidx[k] = (int)(((int64_t)2 * k + 1) * n_pairs / (2 * (int64_t)n_judge));
    is_judged[jidx[k]] = 1;
  }
  bool net_ok = n_judge > 0 && tol > 0;
  DBuf jw, jrows, jnorm;
  std::vector<double> err(n_judge, 0.0);
  if (n_judge > 0) {
    std::vector<int32_t> jpq(2 * (size_t)n_judge);
    for (int k = 0; k < n_judge; ++k) {
      jpq[2 * k] = pq[2 * jidx[k]];
      jpq[2 * k + 1] = pq[2 * jidx[k] + 1];
    }
    jw.alloc(sizeof(double) * ng * n_judge);
    jrows.alloc(sizeof(int) * n_judge);
    jnorm.alloc(sizeof(double) * 2 * n_judge);
    std::vector<int32_t> jst(n_judge, 0);
    try {
      apply_w_device(s, n_judge, jpq.data(), jw.p, false, nullptr, jst.data());
    } catch (const Fail& f) {
      if (f.st != BSE_ERR_NUMERIC) throw;
      net_ok = false;     // a failed judge pair: its row stays NaN, nothing is accepted
    }
    HIPC(hipMemcpyAsync(jrows.p, jidx.data(), sizeof(int) * n_judge, hipMemcpyHostToDevice, s->stream));
    HIPC(launch_diff_norms(w_dev, jrows.as<int>(), jw.as<double>(), n_judge, ng, jnorm.as<double>(), s->stream));
    std::vector<double> nrm(2 * (size_t)n_judge);
    HIPC(hipMemcpyAsync(nrm.data(), jnorm.p, sizeof(double) * nrm.size(), hipMemcpyDeviceToHost, s->stream));
    HIPC(hipStreamSynchronize(s->stream));
    for (int k = 0; k < n_judge; ++k) {
      err[k] = std::sqrt(nrm[2 * (size_t)k] / nrm[2 * (size_t)k + 1]);
      if (!(err[k] <= tol)) net_ok = false;
    }
    // the judged pairs return their propagated W
    for (int k = 0; k < n_judge; ++k)
      HIPC(hipMemcpyAsync(w_dev + (size_t)jidx[k] * ng, jw.as<double>() + (size_t)k * ng, sizeof(double) * ng,
                          hipMemcpyDeviceToDevice, s->stream));
  }
  // 3. every prediction not kept is replaced by the propagation's W
  std::vector<int32_t> acc(n_pairs, 0), rej;
  std::vector<int> ridx;
  for (int k = 0; k < n_pairs; ++k) {
    if (is_judged[k]) continue;
    if (net_ok && sign_ok[k]) {
      acc[k] = 1;
    } else {
      rej.push_back(pq[2 * k]);
      rej.push_back(pq[2 * k + 1]);
      ridx.push_back(k);
    }
  }
  if (!ridx.empty()) {
    DBuf tmp;
    tmp.alloc(sizeof(double) * ng * ridx.size());
    apply_w_device(s, (int)ridx.size(), rej.data(), tmp.p, false, nullptr, nullptr);
    for (size_t j = 0; j < ridx.size(); ++j)
      HIPC(hipMemcpyAsync(w_dev + (size_t)ridx[j] * ng, tmp.as<double>() + j * ng, sizeof(double) * ng,
                          hipMemcpyDeviceToDevice, s->stream));
  }
  HIPC(hipStreamSynchronize(s->stream));
  if (accepted) std::memcpy(accepted, acc.data(), sizeof(int32_t) * n_pairs);
  if (judged_err && n_judge > 0) std::memcpy(judged_err, err.data(), sizeof(double) * n_judge);
}

#define API_BEGIN try {
#define API_END                 \
  }                             \
  catch (const Fail& f) {       \
    return f.st;                \
  }                             \
  catch (const std::exception& e) { \
    g_err = e.what();           \
    return BSE_ERR_DEVICE;      \
  }                             \
  return BSE_OK;

}  // namespace

extern "C" {

const char* bse_last_error(void) { return g_err.c_str(); }
const char* bse_version(void) { return "libbse 0.1 gfx950"; }

bse_status bse_generate_signs(uint64_t seed, int32_t n_stoch, int32_t n_occ, int8_t* xi) {
  if (n_stoch <= 0 || n_occ <= 0 || !xi) {
    g_err = "bse_generate_signs: bad arguments";
    return BSE_ERR_ARG;
  }
  bse_host::stochastic_signs(seed, n_stoch, n_occ, xi);
  return BSE_OK;
}

bse_status bse_create_system(const bse_config* cfg, const double* v_ext, bse_system** out) {
  API_BEGIN
  if (!cfg || !v_ext || !out) fail(BSE_ERR_ARG, "null argument");
  *out = nullptr;
  const bse_config& c = *cfg;
  if (c.nx != c.ny || c.nx != c.nz) fail(BSE_ERR_ARG, "grid must be cubic (nx == ny == nz)");
  const bool fp64 = c.precision == BSE_FP64;
  if (c.precision != BSE_FP64 && c.precision != BSE_MIXED) fail(BSE_ERR_ARG, "bad precision");
  if (fp64 ? !grid_supported<double>(c.nx) : !grid_supported<float>(c.nx))
    fail(BSE_ERR_ARG, "unsupported grid size " + std::to_string(c.nx));
  if (!(c.h > 0) || !(c.dt > 0) || c.n_steps < 0 || c.n_occ <= 0 || c.n_stoch < 0 ||
      c.clean_every < 0 || !(c.gamma >= 0) || c.max_batch < 1)
    fail(BSE_ERR_ARG, "bad configuration value");
  if (c.alpha != 0.0) fail(BSE_ERR_ARG, "only the linearised kick (alpha = 0) is implemented");
  int ndev = 0;
  HIPC(hipGetDeviceCount(&ndev));
  if (c.device < 0 || c.device >= ndev) fail(BSE_ERR_ARG, "bad device ordinal");
  HIPC(hipSetDevice(c.device));
  init_scratch(c.device);
  auto* s = new bse_system();
  try {
    s->cfg = c;
    s->n = c.nx;
    s->ng = (size_t)c.nx * c.ny * c.nz;
    s->dv = c.h * c.h * c.h;
    s->deterministic = c.n_stoch == 0;
    s->L = s->deterministic ? c.n_occ : c.n_stoch;
    s->vext.assign(v_ext, v_ext + s->ng);
    for (double v : s->vext)
      if (!std::isfinite(v)) fail(BSE_ERR_ARG, "non-finite V_ext");
    upload_tables<double>(s, s->td);
    if (!fp64) upload_tables<float>(s, s->tf);
    configure_kernels<double>(s->n);
    if (!fp64) configure_kernels<float>(s->n);
    compute_weights(s);
    if (!s->deterministic) {
      s->xi.resize((size_t)s->L * c.n_occ);
      bse_generate_signs(c.seed, s->L, c.n_occ, s->xi.data());
    }
  } catch (...) {
    delete s;
    throw;
  }
  *out = s;
  API_END
}

bse_status bse_set_signs(bse_system* s, int32_t n_stoch, int32_t n_occ, const int8_t* xi) {
  API_BEGIN
  if (!s || !xi) fail(BSE_ERR_ARG, "null argument");
  if (s->deterministic || n_stoch != s->L || n_occ != s->cfg.n_occ)
    fail(BSE_ERR_ARG, "sign shape does not match the configuration");
  for (size_t i = 0; i < (size_t)n_stoch * n_occ; ++i)
    if (xi[i] != 1 && xi[i] != -1) fail(BSE_ERR_ARG, "signs must be +1 or -1");
  s->xi.assign(xi, xi + (size_t)n_stoch * n_occ);
  s->signs_given = true;
  API_END
}

bse_status bse_set_stream(bse_system* s, void* st) {
  API_BEGIN
  if (!s) fail(BSE_ERR_ARG, "null system");
  s->stream = reinterpret_cast<hipStream_t>(st);
  API_END
}

bse_status bse_set_orbitals(bse_system* s, int32_t n_orb, const double* phi, const double* eps) {
  API_BEGIN
  if (!s || !phi || !eps) fail(BSE_ERR_ARG, "null argument");
  if (n_orb < s->cfg.n_occ) fail(BSE_ERR_ARG, "n_orb < n_occ");
  const size_t tot = (size_t)n_orb * s->ng;
  for (size_t i = 0; i < tot; ++i)
    if (!std::isfinite(phi[i])) fail(BSE_ERR_ARG, "non-finite orbital value");
  for (int i = 0; i < n_orb; ++i)
    if (!std::isfinite(eps[i])) fail(BSE_ERR_ARG, "non-finite eigenvalue");
  HIPC(hipSetDevice(s->cfg.device));
  s->ready = false;
  s->n_orb = n_orb;
  s->eps.assign(eps, eps + n_orb);
  s->mx_eps_v0 = -1;
  s->phi64.alloc(sizeof(double) * tot);
  HIPC(hipMemcpy(s->phi64.p, phi, sizeof(double) * tot, hipMemcpyHostToDevice));
  if (s->cfg.precision == BSE_MIXED) {
    const size_t no = (size_t)s->cfg.n_occ * s->ng;
    s->phi_occ32.alloc(sizeof(float) * no);
    HIPC(launch_to_real<float>(s->phi64.as<double>(), no, s->phi_occ32.as<float>(), s->stream));
    const size_t nt = (size_t)clean_sp(s->cfg.n_occ) * s->ng;
    s->phih.alloc(sizeof(unsigned short) * no);
    s->phil.alloc(sizeof(unsigned short) * no);
    s->phith.alloc(sizeof(unsigned short) * nt);
    s->phitl.alloc(sizeof(unsigned short) * nt);
    HIPC(launch_phi_split(s->phi_occ32.as<float>(), s->cfg.n_occ, s->ng,
                          PhiSplitBufs{s->phih.as<unsigned short>(), s->phil.as<unsigned short>(),
                                       s->phith.as<unsigned short>(), s->phitl.as<unsigned short>()},
                          s->stream));
    prepare_unperturbed<float>(s);
  } else {
    prepare_unperturbed<double>(s);
  }
  HIPC(hipStreamSynchronize(s->stream));
  s->a_no = s->a_nc = 0;
  s->ready = true;
  API_END
}

bse_status bse_apply_W_device(bse_system* s, int32_t n_pairs, const int32_t* pq_dev, void* w_dev,
                              int32_t dtype) {
  API_BEGIN
  check_ready(s);
  if (n_pairs < 0 || (n_pairs > 0 && (!pq_dev || !w_dev))) fail(BSE_ERR_ARG, "bad pair arguments");
  if (dtype != BSE_F64 && dtype != BSE_F32) fail(BSE_ERR_ARG, "dtype must be BSE_F64 or BSE_F32");
  if (n_pairs == 0) return BSE_OK;
  // the indices are read back (after the work already on the stream) and
  // checked before anything is written
  std::vector<int32_t> pq(2 * (size_t)n_pairs);
  HIPC(hipMemcpyAsync(pq.data(), pq_dev, sizeof(int32_t) * pq.size(), hipMemcpyDeviceToHost, s->stream));
  HIPC(hipStreamSynchronize(s->stream));
  check_pairs(s, n_pairs, pq.data());
  apply_w_device(s, n_pairs, pq.data(), w_dev, dtype == BSE_F32, nullptr, nullptr);
  API_END
}

bse_status bse_inject_fault(bse_system* s, int32_t target, int32_t index, int64_t point, double value) {
  API_BEGIN
  check_ready(s);
  if (target != BSE_FAULT_ORBITAL && target != BSE_FAULT_UNPERTURBED) fail(BSE_ERR_ARG, "bse_inject_fault: bad target");
  const int count = target == BSE_FAULT_ORBITAL ? s->n_orb : s->L;
  if (index < 0 || index >= count || point < 0 || (size_t)point >= s->ng)
    fail(BSE_ERR_ARG, "bse_inject_fault: index or point out of range");
  HIPC(hipStreamSynchronize(s->stream));
  if (target == BSE_FAULT_ORBITAL) {
    HIPC(hipMemcpy(s->phi64.as<double>() + (size_t)index * s->ng + point, &value, sizeof(double),
                   hipMemcpyHostToDevice));
  } else if (s->cfg.precision == BSE_FP64) {
    HIPC(hipMemcpy(s->h0.as<cplx<double>>() + (size_t)index * s->ng + point, &value, sizeof(double),
                   hipMemcpyHostToDevice));
  } else {
    const float v = (float)value;
    HIPC(hipMemcpy(s->h0.as<cplx<float>>() + (size_t)index * s->ng + point, &v, sizeof(float),
                   hipMemcpyHostToDevice));
  }
  API_END
}

bse_status bse_apply_W(bse_system* s, int32_t n_pairs, const int32_t* pq, double* w_out,
                       double* wpol_out, int32_t* pair_status) {
  API_BEGIN
  check_ready(s);
  if (n_pairs < 0 || (n_pairs > 0 && (!pq || !w_out))) fail(BSE_ERR_ARG, "bad pair arguments");
  if (n_pairs == 0) return BSE_OK;
  DBuf w, wp;
  const size_t cnt = (size_t)n_pairs * s->ng;
  w.alloc(sizeof(double) * cnt);
  if (wpol_out) wp.alloc(sizeof(double) * cnt);
  std::vector<int32_t> st(n_pairs, 0);
  bse_status rc = BSE_OK;
  try {
    apply_w_device(s, n_pairs, pq, w.p, false, wpol_out ? wp.as<double>() : nullptr, st.data());
  } catch (const Fail& f) {
    if (f.st != BSE_ERR_NUMERIC) throw;
    rc = BSE_ERR_NUMERIC;
  }
  HIPC(hipMemcpyAsync(w_out, w.p, sizeof(double) * cnt, hipMemcpyDeviceToHost, s->stream));
  if (wpol_out)
    HIPC(hipMemcpyAsync(wpol_out, wp.p, sizeof(double) * cnt, hipMemcpyDeviceToHost, s->stream));
  HIPC(hipStreamSynchronize(s->stream));
  if (pair_status) std::memcpy(pair_status, st.data(), sizeof(int32_t) * n_pairs);
  if (rc != BSE_OK) {
    g_err = "non-finite W for some pairs";
    return rc;
  }
  API_END
}

bse_status bse_set_timing(bse_system* s, int32_t enable) {
  API_BEGIN
  if (!s) fail(BSE_ERR_ARG, "null system");
  if (enable < 0 || enable > 2) fail(BSE_ERR_ARG, "bse_set_timing: level 0, 1 or 2");
  HIPC(hipStreamSynchronize(s->stream));
  s->timer.on = enable != 0;
  s->timer.level = enable;
  s->timer.reset();
  API_END
}

bse_status bse_set_yz_schedule(bse_system* s, int32_t schedule) {
  API_BEGIN
  if (!s) fail(BSE_ERR_ARG, "null system");
  if (schedule < 0 || schedule > 2) fail(BSE_ERR_ARG, "bse_set_yz_schedule: schedule 0, 1 or 2");
  HIPC(hipStreamSynchronize(s->stream));
  s->yz_schedule = schedule;
  API_END
}

bse_status bse_set_launch_order(bse_system* s, int32_t order) {
  API_BEGIN
  if (!s) fail(BSE_ERR_ARG, "null system");
  if (order < 0 || order > 7) fail(BSE_ERR_ARG, "bse_set_launch_order: order 0..7");
  HIPC(hipStreamSynchronize(s->stream));
  s->launch_order = order;
  API_END
}

bse_status bse_set_lanczos_path(bse_system* s, int32_t path) {
  API_BEGIN
  if (!s) fail(BSE_ERR_ARG, "null system");
  if (path < 0 || path > 1) fail(BSE_ERR_ARG, "bse_set_lanczos_path: path 0 or 1");
  s->lz_path = path;
  API_END
}

int32_t bse_kernel_times(bse_system* s, int32_t cap, const char** names, double* avg_ms,
                         int32_t* calls) {
  if (!s || !s->timer.on) return 0;
  try {
    HIPC(hipStreamSynchronize(s->stream));
    int k = 0;
    for (const auto& nm : s->timer.order) {
      if (k >= cap) break;
      const auto& r = s->timer.recs[nm];
      double tot = 0;
      for (size_t i = 0; i < r.used; ++i) {
        float ms = 0;
        HIPC(hipEventElapsedTime(&ms, r.ev[i].first, r.ev[i].second));
        tot += ms;
      }
      names[k] = s->timer.recs.find(nm)->first.c_str();
      avg_ms[k] = r.used ? tot / r.used : 0.0;
      calls[k] = (int32_t)r.used;
      ++k;
    }
    return k;
  } catch (const Fail&) {
    return -1;
  }
}

bse_status bse_build_A(bse_system* s, int32_t n_o, int32_t n_c, double* A) {
  API_BEGIN
  build_a(s, n_o, n_c, A);
  API_END
}

bse_status bse_valence_W(bse_system* s, double* w_out) {
  API_BEGIN
  if (!s || !w_out) fail(BSE_ERR_ARG, "bse_valence_W: null argument");
  if (s->a_no == 0) fail(BSE_ERR_STATE, "bse_valence_W: call bse_build_A first");
  const size_t n_ij = (size_t)s->a_no * (s->a_no + 1) / 2;
  HIPC(hipMemcpyAsync(w_out, s->wij.p, sizeof(double) * n_ij * s->ng, hipMemcpyDeviceToHost, s->stream));
  HIPC(hipStreamSynchronize(s->stream));
  API_END
}

bse_status bse_spectrum(bse_system* s, int32_t n_exc, double* omega, double* dip2, int32_t n_w,
                        const double* w_grid, double sigma_broad, double* sigma) {
  API_BEGIN
  spectrum(s, n_exc, omega, dip2, n_w, w_grid, sigma_broad, sigma);
  API_END
}

bse_status bse_boundary_potential(bse_system* s, double* v_bndry) {
  API_BEGIN
  if (!v_bndry) fail(BSE_ERR_ARG, "bse_boundary_potential: null output");
  *v_bndry = boundary_potential(s);
  API_END
}

bse_status bse_fit_box_correction(int32_t n_box, int32_t n_exc, const double* omega, const double* v_bndry,
                                  double* eps_inv, double* c, double* w_k0) {
  API_BEGIN
  if (const char* msg = bse_host::fit_box_correction(n_box, n_exc, omega, v_bndry, eps_inv, c, w_k0))
    fail(BSE_ERR_ARG, msg);
  API_END
}

bse_status bse_apply_A_mixed(bse_system* s, int32_t n_vec, const double* f, double* af) {
  API_BEGIN
  apply_a_mixed(s, n_vec, f, af);
  API_END
}

bse_status bse_chebyshev_mixed(bse_system* s, int32_t n_mom, double e_min, double e_max, int32_t n_w,
                               const double* w_grid, double sigma_broad, double* sigma,
                               double* residues) {
  API_BEGIN
  chebyshev_mixed(s, n_mom, e_min, e_max, n_w, w_grid, sigma_broad, sigma, residues);
  API_END
}

bse_status bse_chebyshev_spectrum(bse_system* s, int32_t n_mom, double e_min, double e_max,
                                  int32_t n_w, const double* w_grid, double sigma_broad,
                                  double* sigma, double* residues, double* bounds) {
  API_BEGIN
  chebyshev_spectrum(s, n_mom, e_min, e_max, n_w, w_grid, sigma_broad, sigma, residues, bounds);
  API_END
}

bse_status bse_chebyshev_spectrum_noalloc(bse_system* s, int32_t n_mom, double e_min, double e_max,
                                          int32_t n_w, const double* w_grid, double sigma_broad,
                                          double* sigma, double* residues, double* bounds) {
  API_BEGIN
  chebyshev_spectrum_noalloc(s, n_mom, e_min, e_max, n_w, w_grid, sigma_broad, sigma, residues, bounds);
  API_END
}

bse_status bse_exciton_states(bse_system* s, int32_t n_mom, double e_min, double e_max, int32_t n_w,
                              const double* w_list, double sigma_broad, double* f_out, double* dens_out,
                              double* bounds) {
  API_BEGIN
  exciton_states(s, n_mom, e_min, e_max, n_w, w_list, sigma_broad, f_out, dens_out, bounds);
  API_END
}

bse_status bse_exciton_states_mixed(bse_system* s, int32_t n_mom, double e_min, double e_max,
                                    int32_t n_w, const double* w_list, double sigma_broad, int32_t n_a,
                                    double* f_out, double* dens_out) {
  API_BEGIN
  exciton_states_mixed(s, n_mom, e_min, e_max, n_w, w_list, sigma_broad, n_a, f_out, dens_out);
  API_END
}

bse_status bse_autotune(bse_system* s, int32_t n_pairs, const char* cache_path) {
  API_BEGIN
  check_ready(s);
  if (n_pairs < 1 || n_pairs > s->cfg.max_batch) fail(BSE_ERR_ARG, "bse_autotune: 1 <= n_pairs <= max_batch");
  if (s->cfg.precision == BSE_FP64) autotune_t<double>(s, n_pairs, cache_path);
  else autotune_t<float>(s, n_pairs, cache_path);
  API_END
}

int32_t bse_tuned_shape(bse_system* s, int32_t* tc, int32_t* nt) {
  if (!s || !tc || !nt) return BSE_ERR_ARG;
  *tc = s->tune_tc;
  *nt = s->tune_nt;
  return BSE_OK;
}

bse_status bse_apply_W_batch(int32_t n_sys, bse_system* const* systems, const int32_t* n_pairs,
                             const int32_t* const* pq, void* const* w_dev, int32_t mode) {
  API_BEGIN
  apply_w_batch(n_sys, systems, n_pairs, pq, w_dev, mode);
  API_END
}

bse_status bse_batch_plan_create(int32_t n_sys, bse_system* const* systems, const int32_t* n_pairs,
                                 const int32_t* const* pq, void* const* w_dev, bse_batch_plan** plan) {
  API_BEGIN
  if (plan) *plan = nullptr;
  plan_create(n_sys, systems, n_pairs, pq, w_dev, plan);
  API_END
}

bse_status bse_batch_plan_run(bse_batch_plan* plan) {
  API_BEGIN
  plan_run(plan);
  API_END
}

void bse_batch_plan_destroy(bse_batch_plan* plan) {
  if (!plan) return;
  (void)hipSetDevice(plan->device);
  (void)hipStreamSynchronize(plan->origin);
  delete plan;
}

bse_status bse_fno_make_samples(bse_system* s, int32_t n_pairs, const int32_t* pq, void* x_dev,
                                void* t_dev, void* scale_dev) {
  API_BEGIN
  make_samples(s, n_pairs, pq, reinterpret_cast<float*>(x_dev), reinterpret_cast<float*>(t_dev),
               reinterpret_cast<double*>(scale_dev));
  API_END
}

bse_status bse_apply_W_surrogate(bse_system* s, bse_fno* net, int32_t n_pairs, const int32_t* pq,
                                 void* w_dev, double tol, int32_t n_judge, int32_t* accepted,
                                 double* judged_err) {
  API_BEGIN
  apply_w_surrogate(s, net, n_pairs, pq, reinterpret_cast<double*>(w_dev), tol, n_judge, accepted, judged_err);
  API_END
}

void bse_destroy_system(bse_system* s) {
  if (!s) return;
  (void)hipSetDevice(s->cfg.device);
  if (s->own_stream) (void)hipStreamDestroy(s->own_stream);
  delete s;
}

}  // extern "C"
