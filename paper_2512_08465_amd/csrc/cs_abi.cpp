// Host runtime and C-ABI of the screening library.
//
// A call screens its outage list through B resident scenario slots (B from
// the HBM budget) that are refilled as scenarios finish.  Two HIP streams:
//   interior-point stream: refill free slots -> islands -> setup, and one
//     Newton step per round for every iterating slot (OPF evaluate/assemble
//     -> KKT LU + solve -> step), then a count of the slots per stage;
//   dynamic stream: for the slots that left the OPF loop, claimed in one
//     step: dynamic Jacobians -> LU + solve (g_y^{-1} g_x) -> state matrix ->
//     Hessenberg + QR -> classify, which writes the record and frees the slot.
// The two overlap: the eigenvalue work of early finishers runs beside the
// Newton steps of the slow scenarios and of the next ones.  One risk
// reduction over the whole list closes the call.  The network is resident on
// the device from cs_net_create; per-call workspace is cached in the context
// and grown when a larger network or batch needs it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <set>
#include <thread>
#include <string>
#include <vector>

#include "../../include/cs.h"
#include "cs_internal.h"

namespace cs {
size_t lu_lds_bytes(int n, int nrhs);
int lu_max_order();
int lu_reg_order();
int lu_reg_order_w4();
int lu_reg_waves(int n, bool f32);
size_t opf_eval_lds(int nb, int nl, int ng);
size_t form_state_lds(int ng);
void lu_set_attrs(size_t bytes);
void opf_set_attrs(size_t bytes);
void dyn_set_attrs(size_t bytes);
void eig_set_attrs(size_t bytes);
constexpr size_t kLdsMax = 160 * 1024;
constexpr int kRefineMax = 4;     // default FP64 refinement steps of a mixed-precision solve
}  // namespace cs

using namespace cs;

static thread_local std::string g_err;
static size_t set_kernel_attrs(int device);

// Scenario workspace of cs_screen_device_noalloc: a static device array, one
// per GPU the library runs on, held until the process ends.  Its address on a
// device comes from hipGetSymbolAddress at cs_ctx_create (the name itself is
// a host-side stand-in and is never passed to a kernel).
static __device__ __align__(256) unsigned char scratch[CS_NOALLOC_SCRATCH_BYTES];

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                        \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess)                                                   \
      return fail(CS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct cs_ctx {
  int device = 0;
  size_t hbm_budget = 0;
  hipStream_t stream = nullptr;
  hipStream_t stream_dyn = nullptr;     // dynamic stage of the screening loop
  hipEvent_t ev_ipm = nullptr, ev_dyn = nullptr;   // cross-stream order (no timing)
  int* d_counter = nullptr;
  int* h_counter = nullptr;
  int* d_sched = nullptr;               // [0..1] next scenario (64-bit), [2..] stage counts
  int* h_sched = nullptr;
  std::vector<hipEvent_t> ev_pool;      // timing events, reused across calls
  int* d_units = nullptr;               // per-launch solve counts when timing
  size_t units_cap = 0;
  // cached workspace
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // kernel timing
  cs_stats stats{};
  size_t lds_max = 64 * 1024;   // dynamic LDS per workgroup this device allows
  int n_cu = 0;                 // compute units of the device
  void* scratch = nullptr;      // this device's copy of the static scratch array
};

// Launch timing: events around each launch on its own stream, resolved when
// the call ends (no synchronisation in between, so the two streams keep
// overlapping).  units = work items of the launch, either known on the host
// or counted on the device into d_units[uidx].
struct TimedLaunches {
  cs_ctx* c;
  bool on;
  struct Rec { int kind; hipEvent_t a, b; int64_t units; int uidx; };
  std::vector<Rec> recs;
  size_t next_ev = 0;
  int n_units = 0;
  TimedLaunches(cs_ctx* c_, bool on_) : c(c_), on(on_) {}
  hipEvent_t ev() {
    if (next_ev == c->ev_pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      c->ev_pool.push_back(e);
    }
    return c->ev_pool[next_ev++];
  }
  // a device slot for a unit count, or -1 when timing is off / full
  int unit_slot() {
    if (!on || (size_t)n_units >= c->units_cap) return -1;
    return n_units++;
  }
  template <class F>
  int run(int kind, hipStream_t st, int64_t units, int uidx, F launch) {
    hipEvent_t a = nullptr, b = nullptr;
    if (on) {
      a = ev();
      b = ev();
      if (!a || !b || hipEventRecord(a, st) != hipSuccess) return fail(CS_EDEVICE, "timing event failed");
    }
    launch();
    if (on) {
      if (hipEventRecord(b, st) != hipSuccess) return fail(CS_EDEVICE, "timing event failed");
      recs.push_back(Rec{kind, a, b, units, uidx});
    }
    return CS_OK;
  }
  // after both streams have drained
  int resolve() {
    if (!on) return CS_OK;
    std::vector<int> u(n_units);
    if (n_units && hipMemcpy(u.data(), c->d_units, sizeof(int) * n_units,
                             hipMemcpyDeviceToHost) != hipSuccess)
      return fail(CS_EDEVICE, "timing counts copy failed");
    for (const Rec& r : recs) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
        return fail(CS_EDEVICE, "timing event query failed");
      c->stats.ms[r.kind] += ms;
      c->stats.launches[r.kind] += 1;
      c->stats.units[r.kind] += (r.uidx >= 0) ? u[r.uidx] : r.units;
    }
    return CS_OK;
  }
};

struct cs_net {
  cs_ctx* ctx = nullptr;
  int device = 0;       // kept here so that destroying never reads the context
  DevNet d{};
  std::vector<void*> allocs;
  int nb = 0, nl = 0, ng = 0, nd = 0;
  int na = 0;           // largest state-matrix order: 7 per machine + 8 per converter - 1
};

// Raise the dynamic LDS limit of the kernels that need more than the
// default to what the device allows; returns that limit.  Errors are cleared
// so they do not surface in a later, unrelated runtime call.
static size_t set_kernel_attrs(int device) {
  int per_block = 0, optin = 0;
  hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
  hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, device);
  size_t lim = (size_t)std::max(per_block, optin);
  lim = std::min(lim, kLdsMax);
  if (lim > 64 * 1024) {
    lu_set_attrs(lim);
    opf_set_attrs(lim);
    dyn_set_attrs(lim);
    eig_set_attrs(lim);
  }
  (void)hipGetLastError();
  return lim;
}

extern "C" {

const char* cs_last_error(void) { return g_err.c_str(); }
int cs_abi_version(void) { return CS_ABI_VERSION; }

void cs_opts_default(cs_opts* o) {
  if (!o) return;
  o->prec = CS_PREC_FP64;
  o->max_it = 150;
  o->tol = 1e-8;
  o->near_eps = 1e-6;
  o->hbm_budget = 0;
  o->batch = 0;
  o->timing = 0;
  o->overlap = 0;
  o->refine_steps = kRefineMax;
  o->graph = 0;
  o->autotune = 0;
}

int cs_ctx_create(int device, size_t hbm_budget, cs_ctx** out) {
  if (!out) return fail(CS_EINVAL, "cs_ctx_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev)
    return fail(CS_EINVAL, "cs_ctx_create: device " + std::to_string(device) +
                               " out of range (" + std::to_string(ndev) + " devices)");
  HIPCHK(hipSetDevice(device));
  cs_ctx* c = new cs_ctx();
  c->device = device;
  c->hbm_budget = hbm_budget ? hbm_budget : ((size_t)48 << 30);
  // both streams at the default priority
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&c->stream_dyn, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_ipm, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_dyn, hipEventDisableTiming) != hipSuccess ||
      hipMalloc(&c->d_counter, sizeof(int)) != hipSuccess ||
      hipHostMalloc(&c->h_counter, sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipMalloc(&c->d_sched, sizeof(int) * (PH_COUNT + 3)) != hipSuccess ||
      hipHostMalloc(&c->h_sched, sizeof(int) * (PH_COUNT + 3), hipHostMallocDefault) != hipSuccess) {
    cs_ctx_destroy(c);
    return fail(CS_EDEVICE, "cs_ctx_create: stream or counter allocation failed");
  }
  // kernels whose LDS may exceed the default dynamic limit
  c->lds_max = set_kernel_attrs(device);
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    c->n_cu = 0;
  // the device address of the static scratch array on this device
  const hipError_t se = hipGetSymbolAddress(&c->scratch, HIP_SYMBOL(scratch));
  if (se != hipSuccess || c->scratch == nullptr) {
    cs_ctx_destroy(c);
    return fail(CS_EDEVICE, std::string("cs_ctx_create: scratch address: ") + hipGetErrorString(se));
  }
  *out = c;
  return CS_OK;
}

void cs_ctx_destroy(cs_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  if (c->ws) hipFree(c->ws);
  if (c->d_counter) hipFree(c->d_counter);
  if (c->h_counter) hipHostFree(c->h_counter);
  if (c->d_sched) hipFree(c->d_sched);
  if (c->h_sched) hipHostFree(c->h_sched);
  if (c->d_units) hipFree(c->d_units);
  if (c->stream) hipStreamDestroy(c->stream);
  if (c->stream_dyn) hipStreamDestroy(c->stream_dyn);
  if (c->ev_ipm) hipEventDestroy(c->ev_ipm);
  if (c->ev_dyn) hipEventDestroy(c->ev_dyn);
  for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
  delete c;
}

int cs_stats_get(const cs_ctx* c, cs_stats* out) {
  if (!c || !out) return fail(CS_EINVAL, "cs_stats_get: NULL argument");
  *out = c->stats;
  return CS_OK;
}

int cs_stats_reset(cs_ctx* c) {
  if (!c) return fail(CS_EINVAL, "cs_stats_reset: NULL argument");
  c->stats = cs_stats{};
  return CS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ network
template <class T>
static int upload(cs_net* n, const T* host, size_t count, const T** dst) {
  void* p = nullptr;
  const size_t bytes = std::max<size_t>(1, count) * sizeof(T);
  if (hipMalloc(&p, bytes) != hipSuccess) return fail(CS_ENOMEM, "device allocation failed");
  n->allocs.push_back(p);
  if (count && hipMemcpy(p, host, count * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return fail(CS_EDEVICE, "host to device copy failed");
  *dst = static_cast<const T*>(p);
  return CS_OK;
}

static bool all_finite(const double* a, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

extern "C" void cs_net_destroy(cs_net* n) {
  if (!n) return;
  hipSetDevice(n->device);
  for (void* p : n->allocs) hipFree(p);
  delete n;
}

extern "C" int cs_net_create(cs_ctx* ctx, const cs_net_desc* d, cs_net** out) {
  if (!ctx || !d || !out) return fail(CS_EINVAL, "cs_net_create: NULL argument");
  *out = nullptr;
  const int nb = d->n_bus, nl = d->n_branch, ng = d->n_gen, nd = d->n_load;
  if (nb <= 0 || nl < 0 || ng <= 0 || nd < 0)
    return fail(CS_EINVAL, "cs_net_create: sizes must be n_bus > 0, n_gen > 0, others >= 0");
  int n_states = 0;
  for (int g = 0; g < ng; ++g) n_states += (d->gen_kind && d->gen_kind[g] == 1) ? 8 : 7;
  if (nb > 4096 || ng > 1024 || n_states - 1 > 1024)
    return fail(CS_EUNSUPPORTED, "cs_net_create: at most 4096 buses and 1024 dynamic states");
  if (d->ref_bus < 0 || d->ref_bus >= nb) return fail(CS_EINVAL, "cs_net_create: ref_bus out of range");
  if (!(d->base_mva > 0) || !(d->f_hz > 0)) return fail(CS_EINVAL, "cs_net_create: base_mva and f_hz must be > 0");
  const double* need[] = {d->vmin, d->vmax, d->gs, d->bs, d->br_r, d->br_x, d->br_b, d->br_rate,
                          d->pmin, d->pmax, d->qmin, d->qmax, d->c2, d->c1, d->c0, d->dyn, d->pd, d->qd};
  for (const double* p : need)
    if (!p) return fail(CS_EINVAL, "cs_net_create: a required array is NULL");
  if (!d->br_from || !d->br_to || !d->gen_bus || (nd && !d->load_bus))
    return fail(CS_EINVAL, "cs_net_create: an index array is NULL");
  if (!all_finite(d->vmin, nb) || !all_finite(d->vmax, nb) || !all_finite(d->gs, nb) ||
      !all_finite(d->bs, nb) || !all_finite(d->br_r, nl) || !all_finite(d->br_x, nl) ||
      !all_finite(d->br_b, nl) || !all_finite(d->br_rate, nl) || !all_finite(d->pmin, ng) ||
      !all_finite(d->pmax, ng) || !all_finite(d->qmin, ng) || !all_finite(d->qmax, ng) ||
      !all_finite(d->c2, ng) || !all_finite(d->c1, ng) || !all_finite(d->c0, ng) ||
      !all_finite(d->dyn, ng * CS_N_DYN) || !all_finite(d->pd, nd) || !all_finite(d->qd, nd))
    return fail(CS_EINVAL, "cs_net_create: non-finite value in the network");
  for (int l = 0; l < nl; ++l) {
    if (d->br_from[l] < 0 || d->br_from[l] >= nb || d->br_to[l] < 0 || d->br_to[l] >= nb)
      return fail(CS_EINVAL, "cs_net_create: branch " + std::to_string(l) + " bus out of range");
    if (d->br_from[l] == d->br_to[l])
      return fail(CS_EINVAL, "cs_net_create: branch " + std::to_string(l) + " is a self-loop");
    if (d->br_r[l] == 0.0 && d->br_x[l] == 0.0)
      return fail(CS_EINVAL, "cs_net_create: branch " + std::to_string(l) + " has zero impedance");
  }
  for (int b = 0; b < nb; ++b)
    if (!(d->vmin[b] > 0) || d->vmin[b] > d->vmax[b])
      return fail(CS_EINVAL, "cs_net_create: bus " + std::to_string(b) + " needs 0 < vmin <= vmax");
  for (int g = 0; g < ng; ++g) {
    if (d->gen_bus[g] < 0 || d->gen_bus[g] >= nb)
      return fail(CS_EINVAL, "cs_net_create: generator " + std::to_string(g) + " bus out of range");
    const int kind = d->gen_kind ? d->gen_kind[g] : 0;
    if (kind != 0 && kind != 1)
      return fail(CS_EUNSUPPORTED, "cs_net_create: generator kinds 0 (synchronous) and 1 "
                                   "(grid-following converter) only");
    if (d->pmin[g] > d->pmax[g] || d->qmin[g] > d->qmax[g])
      return fail(CS_EINVAL, "cs_net_create: generator " + std::to_string(g) + " has min > max");
    const double* p = d->dyn + (size_t)g * CS_N_DYN;
    if (kind == 0) {
      // H, Td0', Tq0', TA, R, Tg, Tt appear as divisors
      if (!(p[0] > 0) || !(p[6] > 0) || !(p[7] > 0) || !(p[10] > 0) || !(p[11] > 0) ||
          !(p[12] > 0) || !(p[13] > 0))
        return fail(CS_EINVAL, "cs_net_create: generator " + std::to_string(g) +
                                   " needs positive H, Td0', Tq0', TA, R, Tg, Tt");
    } else {
      // Kic, Lf, Cdc, Kidc, Vdc0 appear as divisors
      if (!(p[3] > 0) || !(p[4] > 0) || !(p[6] > 0) || !(p[8] > 0) || !(p[9] > 0))
        return fail(CS_EINVAL, "cs_net_create: converter " + std::to_string(g) +
                                   " needs positive Kic, Lf, Cdc, Kidc, Vdc0");
    }
  }
  for (int k = 0; k < nd; ++k)
    if (d->load_bus[k] < 0 || d->load_bus[k] >= nb)
      return fail(CS_EINVAL, "cs_net_create: load " + std::to_string(k) + " bus out of range");

  {
    const size_t nk = 4 * (size_t)nb + 2 * (size_t)ng;
    const size_t lim = ctx->lds_max;
    const int ny = 2 * ng + 2 * nb;
    if ((int)nk > lu_max_order() || ny > lu_max_order() ||
        lu_lds_bytes((int)nk, 1) > lim || lu_lds_bytes(ny, 3 * ng) > lim ||
        opf_eval_lds(nb, nl, ng) > lim ||
        form_state_lds(ng) > lim || 8 * (size_t)(2 * nl + 2 * nb + 4 * ng) > lim)
      return fail(CS_EUNSUPPORTED, "cs_net_create: network too large for the on-chip working set (KKT order " +
                                       std::to_string(nk) + ", " + std::to_string(lim) +
                                       " bytes of LDS per workgroup)");
  }
  HIPCHK(hipSetDevice(ctx->device));
  cs_net* n = new cs_net();
  n->ctx = ctx;
  n->device = ctx->device;
  n->nb = nb; n->nl = nl; n->ng = ng; n->nd = nd;
  n->na = n_states - 1;
  std::vector<int> kinds(ng, 0);
  if (d->gen_kind)
    for (int g = 0; g < ng; ++g) kinds[g] = d->gen_kind[g];
  // branch admittances (pi model, tap and shift on the from side)
  std::vector<double> yffr(nl), yffi(nl), yftr(nl), yfti(nl), ytfr(nl), ytfi(nl), yttr(nl), ytti(nl);
  for (int l = 0; l < nl; ++l) {
    const double r = d->br_r[l], x = d->br_x[l], b = d->br_b[l];
    const double den = r * r + x * x;
    const double ys_r = r / den, ys_i = -x / den;
    double tap = d->br_tap ? d->br_tap[l] : 1.0;
    if (tap == 0.0) tap = 1.0;
    const double sh = d->br_shift ? d->br_shift[l] : 0.0;
    const double cr = tap * std::cos(sh), ci = tap * std::sin(sh);  // t e^{j phi}
    yttr[l] = ys_r;
    ytti[l] = ys_i + 0.5 * b;
    yffr[l] = yttr[l] / (tap * tap);
    yffi[l] = ytti[l] / (tap * tap);
    // Yft = -ys / conj(t e^{j phi}),  Ytf = -ys / (t e^{j phi})
    const double t2 = cr * cr + ci * ci;
    // -ys / (cr - j ci) = -ys (cr + j ci) / t2
    yftr[l] = -(ys_r * cr - ys_i * ci) / t2;
    yfti[l] = -(ys_r * ci + ys_i * cr) / t2;
    // -ys / (cr + j ci) = -ys (cr - j ci) / t2
    ytfr[l] = -(ys_r * cr + ys_i * ci) / t2;
    ytfi[l] = -(ys_i * cr - ys_r * ci) / t2;
  }
  // CSR incidence, ascending ids within each bus
  auto csr = [&](int nitems, auto bus_of, std::vector<int>& ptr, std::vector<int>& idx) {
    ptr.assign(nb + 1, 0);
    for (int i = 0; i < nitems; ++i) bus_of(i, [&](int b) { ptr[b + 1]++; });
    for (int b = 0; b < nb; ++b) ptr[b + 1] += ptr[b];
    idx.assign(ptr[nb], 0);
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (int i = 0; i < nitems; ++i) bus_of(i, [&](int b) { idx[fill[b]++] = i; });
  };
  std::vector<int> bbp, bbi, bgp, bgi, blp, bli;
  csr(nl, [&](int l, auto add) { add(d->br_from[l]); add(d->br_to[l]); }, bbp, bbi);
  csr(ng, [&](int g, auto add) { add(d->gen_bus[g]); }, bgp, bgi);
  csr(nd, [&](int k, auto add) { add(d->load_bus[k]); }, blp, bli);
  std::vector<double> rate(d->br_rate, d->br_rate + nl);
  int rc = CS_OK;
  DevNet& D = n->d;
  D.nb = nb; D.nl = nl; D.ng = ng; D.nd = nd; D.ref_bus = d->ref_bus;
  D.base_mva = d->base_mva;
  D.ws = 2.0 * M_PI * d->f_hz;
#define UP(ptr, cnt, dst) if (rc == CS_OK) rc = upload(n, ptr, cnt, &dst)
  UP(d->br_from, nl, D.br_f); UP(d->br_to, nl, D.br_t);
  UP(yffr.data(), nl, D.yff_re); UP(yffi.data(), nl, D.yff_im);
  UP(yftr.data(), nl, D.yft_re); UP(yfti.data(), nl, D.yft_im);
  UP(ytfr.data(), nl, D.ytf_re); UP(ytfi.data(), nl, D.ytf_im);
  UP(yttr.data(), nl, D.ytt_re); UP(ytti.data(), nl, D.ytt_im);
  UP(rate.data(), nl, D.rate);
  UP(d->vmin, nb, D.vmin); UP(d->vmax, nb, D.vmax); UP(d->gs, nb, D.gs); UP(d->bs, nb, D.bs);
  UP(bbp.data(), nb + 1, D.bus_br_ptr); UP(bbi.data(), bbi.size(), D.bus_br);
  UP(bgp.data(), nb + 1, D.bus_gen_ptr); UP(bgi.data(), bgi.size(), D.bus_gen);
  UP(blp.data(), nb + 1, D.bus_load_ptr); UP(bli.data(), bli.size(), D.bus_load);
  UP(d->gen_bus, ng, D.gen_bus);
  UP(d->pmin, ng, D.pmin); UP(d->pmax, ng, D.pmax); UP(d->qmin, ng, D.qmin); UP(d->qmax, ng, D.qmax);
  UP(d->c2, ng, D.c2); UP(d->c1, ng, D.c1); UP(d->c0, ng, D.c0);
  UP(d->dyn, (size_t)ng * CS_N_DYN, D.dyn);
  UP(kinds.data(), ng, D.gen_kind);
  UP(d->load_bus, nd, D.load_bus); UP(d->pd, nd, D.pd); UP(d->qd, nd, D.qd);
#undef UP
  if (rc != CS_OK) {
    cs_net_destroy(n);
    return rc;
  }
  *out = n;
  return CS_OK;
}

// ---------------------------------------------------------------- workspace
static size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Plan {
  Slots s{};
  size_t per_slot = 0;
};

static Plan plan_sizes(const cs_net* n, bool mixed) {
  Plan p;
  Slots& s = p.s;
  const int nb = n->nb, nl = n->nl, ng = n->ng;
  s.nx = 2 * nb + 2 * ng;
  s.neq = 2 * nb;
  s.nk = s.nx + s.neq;
  s.ldk = (int)round_up(s.nk + 1, 2);      // row stride: matrix + right-hand side
  s.ni = 2 * nl + 2 * nb + 4 * ng;
  s.ny = 2 * ng + 2 * nb;
  s.nyc = s.ny + 3 * ng;
  s.ldy = (int)round_up(s.nyc, 2);
  s.na = n->na;
  s.lda_a = (int)round_up(std::max(s.na, 1), 2);
  // the KKT array also serves as the eigenvalue kernel's scratch
  s.k_stride = round_up(std::max({(size_t)s.nk * s.ldk, (size_t)s.ny * s.ldy,
                                  eig_scratch_doubles(s.na)}), 64);
  s.a_stride = round_up((size_t)s.lda_a * s.na, 64);
  const size_t piv = std::max(s.nk, s.ny);
  p.per_slot = 8 * (s.k_stride + s.a_stride + s.nx + s.neq + 3 * (size_t)s.ni + 8 * (size_t)nl +
                    2 * (size_t)nb +
                    2 * (size_t)s.na) +
               4 * ((size_t)nb + piv + 1) + nb + nl + ng + sizeof(SlotState) + 16 * 64;
  if (mixed) {
    s.ld32 = (int)round_up(s.nk + 1, 4);
    s.k32_stride = round_up((size_t)s.nk * s.ld32, 64);
    p.per_slot += 4 * s.k32_stride;
  } else {
    s.ld32 = 0;
    s.k32_stride = 0;
  }
  return p;
}

// carve the slot arrays out of one allocation.  With fixed != nullptr the
// arrays go into that region of fixed_bytes (nothing is allocated; a layout
// that does not fit fails with CS_EHBM); else into *ws, grown on demand.
static int bind_workspace(void** ws, size_t* ws_bytes, const cs_net* n, Plan& p, int B,
                          void* fixed = nullptr, size_t fixed_bytes = 0) {
  Slots& s = p.s;
  const size_t nb = n->nb, nl = n->nl, ng = n->ng;
  const size_t piv = std::max(s.nk, s.ny);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = round_up(off, 256);
    off = o + bytes;
    return o;
  };
  const size_t oK = take(8 * s.k_stride * B);
  const size_t oA = take(8 * s.a_stride * B);
  const size_t ox = take(8 * (size_t)s.nx * B);
  const size_t ol = take(8 * (size_t)s.neq * B);
  const size_t oz = take(8 * (size_t)s.ni * B);
  const size_t om = take(8 * (size_t)s.ni * B);
  const size_t oh = take(8 * (size_t)s.ni * B);
  const size_t ojh = take(8 * 8 * nl * B + 64);
  const size_t opd = take(8 * nb * B);
  const size_t oqd = take(8 * nb * B);
  const size_t owr = take(8 * (size_t)s.na * B);
  const size_t owi = take(8 * (size_t)s.na * B);
  const size_t olab = take(4 * nb * B);
  const size_t opiv = take(4 * piv * B);
  const size_t obus = take(nb * B);
  const size_t obr = take(nl * B + 64);
  const size_t ogen = take(ng * B + 64);
  const size_t ost = take(sizeof(SlotState) * (size_t)B);
  const size_t ojob = take(4 * ((size_t)B + 2));
  const size_t o32 = take(4 * s.k32_stride * B);
  const size_t need = off;
  char* base = nullptr;
  if (fixed) {
    if (need > fixed_bytes)
      return fail(CS_EHBM, "workspace of " + std::to_string(B) + " slots needs " +
                               std::to_string(need) + " bytes, above the " +
                               std::to_string(fixed_bytes) + " bytes of the scratch region");
    base = static_cast<char*>(fixed);
  } else {
    if (need > *ws_bytes) {
      if (*ws) hipFree(*ws);
      *ws = nullptr;
      *ws_bytes = 0;
      if (hipMalloc(ws, need) != hipSuccess) return fail(CS_ENOMEM, "workspace allocation failed");
      *ws_bytes = need;
    }
    base = static_cast<char*>(*ws);
  }
  s.B = B;
  s.K = reinterpret_cast<double*>(base + oK);
  s.A = reinterpret_cast<double*>(base + oA);
  s.x = reinterpret_cast<double*>(base + ox);
  s.lam = reinterpret_cast<double*>(base + ol);
  s.z = reinterpret_cast<double*>(base + oz);
  s.mu = reinterpret_cast<double*>(base + om);
  s.hv = reinterpret_cast<double*>(base + oh);
  s.jh = reinterpret_cast<double*>(base + ojh);
  s.pd = reinterpret_cast<double*>(base + opd);
  s.qd = reinterpret_cast<double*>(base + oqd);
  s.wr = reinterpret_cast<double*>(base + owr);
  s.wi = reinterpret_cast<double*>(base + owi);
  s.label = reinterpret_cast<int*>(base + olab);
  s.piv = reinterpret_cast<int*>(base + opiv);
  s.bus_on = reinterpret_cast<uint8_t*>(base + obus);
  s.br_on = reinterpret_cast<uint8_t*>(base + obr);
  s.gen_on = reinterpret_cast<uint8_t*>(base + ogen);
  s.st = reinterpret_cast<SlotState*>(base + ost);
  s.jobs = reinterpret_cast<int*>(base + ojob);
  s.K32 = s.k32_stride ? reinterpret_cast<float*>(base + o32) : nullptr;
  return CS_OK;
}


// ------------------------------------------------------------------ engine
// The slot scheduler shared by the batch entry points and the server: B
// slots over a stream of scenarios (a call's list, or a server's ring of
// capacity q_cap), advanced one round at a time.  A round refills free slots,
// takes one Newton step in every iterating slot, counts the slots per stage
// and, when enough have left the OPF loop, claims them for the dynamic stage
// (on the second stream when overlapping).
struct Engine {
  cs_ctx* c = nullptr;
  const DevNet* D = nullptr;
  Slots s{};
  cs_opts opts{};
  int nslots = 0, pstride = 0, dyn_min = 1;
  bool eager = false;            // claim as soon as the OPF tail is shorter (serving)
  hipStream_t st = nullptr, sd = nullptr;
  hipEvent_t ev_ipm = nullptr, ev_dyn = nullptr;
  unsigned long long* d_next = nullptr;
  int* d_counts = nullptr;       // [PH_COUNT]
  int* h_counts = nullptr;       // pinned [PH_COUNT + 1]: stage counts, job-list overflow flag
  unsigned long long* h_next = nullptr;   // pinned
  const int* d_list = nullptr;   // outage pairs
  cs_result* d_res = nullptr;
  long long q_cap = 0;
  const int* item_req = nullptr;
  int* req_done = nullptr;
  const double* load_scale = nullptr;  // serving: [request slot][n_load] factors
  TimedLaunches* T = nullptr;
  const DetailOut* detail = nullptr;   // per-scenario detail (parity entry point)
  int width = 2;                 // ids per outage row (3 for N-3 lists)
  int cnt[PH_COUNT]{};
  long long assigned = 0;        // scenarios handed to slots so far
  bool dyn_busy = false;
  bool dyn_finished = false;     // the dynamic stage was seen complete in issue()
  hipGraphExec_t newton = nullptr;  // captured Newton step (opts.graph > 0)

  Engine() = default;
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;
  ~Engine() {
    if (newton) hipGraphExecDestroy(newton);
  }

  // One Newton step for every slot in the OPF loop, launches only (what the
  // graph captures): KKT assembly, factorisation and solve, update.
  void newton_launches(hipStream_t q) {
    launch_opf_eval(*D, s, nslots, opts.tol, opts.max_it, q);
    if (opts.prec == CS_PREC_MIXED) {
      launch_kkt_to_f32(s, nslots, q);
      launch_lu_solve_f32(s.K32, s.k32_stride, s.nk, s.nk + 1, s.ld32, s.piv, pstride, s.st,
                          PH_IPM, 1, nslots, nullptr, q);
      launch_kkt_refine(s, nslots, pstride, opts.refine_steps, q);
      launch_lu_solve(s.K, s.k_stride, s.nk, s.nk + 1, s.ldk, s.piv, pstride, s.st, PH_IPM, 3,
                      nslots, nullptr, q, LU_KKT_FALLBACK);
    } else {
      launch_lu_solve(s.K, s.k_stride, s.nk, s.nk + 1, s.ldk, s.piv, pstride, s.st, PH_IPM, 1,
                      nslots, nullptr, q);
    }
    launch_opf_update(*D, s, nslots, 1e10, q);
  }

  // opts.graph Newton steps replayed from the captured graph (captured on
  // first use; the kernels read every slot's stage from device memory, so
  // one capture serves every round)
  int newton_graph() {
    if (!newton) {
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      newton_launches(st);
      const hipError_t ec = hipStreamEndCapture(st, &g);
      if (ec != hipSuccess) return fail(CS_EDEVICE, std::string("Newton step capture: ") + hipGetErrorString(ec));
      const hipError_t ei = hipGraphInstantiate(&newton, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (ei != hipSuccess) {
        newton = nullptr;
        return fail(CS_EDEVICE, std::string("Newton step graph: ") + hipGetErrorString(ei));
      }
    }
    for (int r = 0; r < opts.graph; ++r) HIPCHK(hipGraphLaunch(newton, st));
    return CS_OK;
  }

  int timed(int kind, hipStream_t stream, int64_t units, int uidx, const std::function<void()>& f) {
    if (T) return T->run(kind, stream, units, uidx, f);
    f();
    return CS_OK;
  }

  int start() {
    HIPCHK(hipMemsetAsync(s.st, 0, sizeof(SlotState) * (size_t)nslots, st));
    HIPCHK(hipMemsetAsync(s.jobs, 0, 2 * sizeof(int), st));
    HIPCHK(hipMemsetAsync(d_next, 0, sizeof(unsigned long long), st));
    HIPCHK(hipEventRecord(ev_ipm, st));
    HIPCHK(hipStreamWaitEvent(sd, ev_ipm, 0));
    for (int k = 0; k < PH_COUNT; ++k) cnt[k] = 0;
    cnt[PH_EMPTY] = nslots;
    assigned = 0;
    dyn_busy = false;
    return CS_OK;
  }

  int count() {
    launch_phase_counts(s, nslots, d_counts, st);
    HIPCHK(hipMemcpyAsync(h_counts, d_counts, sizeof(int) * PH_COUNT, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_next, d_next, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int k = 0; k < PH_COUNT; ++k) cnt[k] = h_counts[k];
    return CS_OK;
  }

  // One round with N scenarios available so far (absolute count).  idle is
  // set when every available scenario has been recorded and no slot is busy.
  int round(long long N, bool& idle) {
    int rc = issue(N);
    if (rc != CS_OK) return rc;
    return settle(N, idle, true, nullptr);
  }

  // First half of a round, asynchronous: refill, one Newton step, and the
  // stage counts on their way to the host.
  int issue(long long N) {
    bool work = false;
    int rc;
    if (assigned < N && cnt[PH_EMPTY] > 0) {
      const long long nnew = std::min<long long>(cnt[PH_EMPTY], N - assigned);
      rc = timed(CS_K_TOPOLOGY, st, nnew, -1, [&] {
        launch_refill(s, nslots, d_next, N, q_cap, st);
        launch_islands(*D, s, d_list, nslots, st, width);
        launch_setup_k(*D, s, nslots, d_list, st, width, load_scale, item_req);
      });
      if (rc != CS_OK) return rc;
      work = true;
    }
    if ((work || cnt[PH_IPM] > 0) && opts.graph > 0 && !T) {
      if ((rc = newton_graph()) != CS_OK) return rc;
    } else if (work || cnt[PH_IPM] > 0) {
      // At most this many slots are in the OPF loop this step (the LU's
      // launch geometry depends on it): those at the last count and whatever
      // the refill could have added since.  Each per-slot launch of the step
      // runs one workgroup per listed slot, those with work first (at most
      // `grid` of them, checked on the device).
      const long long jobs = (long long)cnt[PH_IPM] + cnt[PH_NEW] + (assigned < N ? N - assigned : 0);
      const int max_jobs = (int)std::min<long long>(jobs, INT_MAX);
      const JobList jl{s.jobs, (int)std::min<long long>(jobs, nslots)};
      launch_job_list(s, nslots, PH_IPM, JOB_ANY, jl.grid, st);
      rc = timed(CS_K_KKT_ASSEMBLE, st, cnt[PH_IPM], -1,
                 [&] { launch_opf_eval(*D, s, nslots, opts.tol, opts.max_it, st, jl); });
      if (rc != CS_OK) return rc;
      const int u = T ? T->unit_slot() : -1;
      if (opts.prec == CS_PREC_MIXED) {
        // (scenarios already on FP64 factorisations are switched to job 3 here)
        launch_job_list(s, nslots, PH_IPM, 1, jl.grid, st);
        rc = timed(CS_K_KKT_REFINE, st, 0, -1, [&] { launch_kkt_to_f32(s, nslots, st, jl); });
        if (rc != CS_OK) return rc;
        if (u >= 0) launch_count_jobs(s, nslots, 1, c->d_units + u, st);
        launch_job_list(s, nslots, PH_IPM, 1, jl.grid, st);
        rc = timed(CS_K_KKT_LU, st, 0, u, [&] {
          launch_lu_solve_f32(s.K32, s.k32_stride, s.nk, s.nk + 1, s.ld32, s.piv, pstride, s.st,
                              PH_IPM, 1, nslots, nullptr, st, jl);
        });
        if (rc != CS_OK) return rc;
        // (the same slots: the factorisation changes no job)
        rc = timed(CS_K_KKT_REFINE, st, 0, -1,
                   [&] { launch_kkt_refine(s, nslots, pstride, opts.refine_steps, st, jl); });
        if (rc != CS_OK) return rc;
        const int u3 = T ? T->unit_slot() : -1;
        if (u3 >= 0) launch_count_jobs(s, nslots, 3, c->d_units + u3, st);
        launch_job_list(s, nslots, PH_IPM, 3, jl.grid, st);
        rc = timed(CS_K_KKT_LU64, st, 0, u3, [&] {
          launch_lu_solve(s.K, s.k_stride, s.nk, s.nk + 1, s.ldk, s.piv, pstride, s.st, PH_IPM, 3,
                          nslots, nullptr, st, LU_KKT_FALLBACK, max_jobs, jl);
        });
      } else {
        if (u >= 0) launch_count_jobs(s, nslots, 1, c->d_units + u, st);
        launch_job_list(s, nslots, PH_IPM, 1, jl.grid, st);
        rc = timed(CS_K_KKT_LU, st, 0, u, [&] {
          launch_lu_solve(s.K, s.k_stride, s.nk, s.nk + 1, s.ldk, s.piv, pstride, s.st, PH_IPM, 1,
                          nslots, nullptr, st, LU_KKT, max_jobs, jl);
        });
      }
      if (rc != CS_OK) return rc;
      launch_job_list(s, nslots, PH_IPM, JOB_NONZERO, jl.grid, st);
      rc = timed(CS_K_IPM_UPDATE, st, cnt[PH_IPM], -1,
                 [&] { launch_opf_update(*D, s, nslots, 1e10, st, jl); });
      if (rc != CS_OK) return rc;
    }
    // Ask whether the dynamic stage has finished before the slot counts are
    // taken: if it finished between the two, its slots would be counted as
    // still busy while it is marked idle, and nothing would free them.
    dyn_finished = false;
    if (dyn_busy) {
      const hipError_t q = hipEventQuery(ev_dyn);
      if (q == hipSuccess) dyn_finished = true;
      else if (q != hipErrorNotReady) return fail(CS_EDEVICE, "dynamic stage failed");
    }
    launch_phase_counts(s, nslots, d_counts, st);
    HIPCHK(hipMemcpyAsync(h_counts, d_counts, sizeof(int) * PH_COUNT, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_next, d_next, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_counts + PH_COUNT, s.jobs + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    return CS_OK;
  }

  // Second half: wait for the counts, then hand finished slots to the
  // dynamic stage.  When the only thing left is to wait for the dynamic
  // stage, a caller that may not block gets *waiting = true instead.
  int settle(long long N, bool& idle, bool may_block, bool* waiting) {
    idle = false;
    if (waiting) *waiting = false;
    int rc;
    HIPCHK(hipStreamSynchronize(st));
    for (int k = 0; k < PH_COUNT; ++k) cnt[k] = h_counts[k];
    if (h_counts[PH_COUNT] != 0)
      return fail(CS_EDEVICE, "internal: a per-slot launch had fewer workgroups than slots with work");
    if (dyn_finished) dyn_busy = false;
    assigned = std::min<long long>((long long)*h_next, N);
    const int ready = cnt[PH_DYN] + cnt[PH_DONE];
    const int ipm_left = cnt[PH_IPM] + cnt[PH_NEW];
    // While more scenarios wait, the dynamic stage takes the ready slots in
    // groups of dyn_min so that they can be refilled.  At the end of a list,
    // one stream waits for the last OPF to finish (one large eigenvalue
    // launch); two streams (overlap 1), or a server, start as soon as the OPF
    // tail is smaller than what waits; overlap 2 starts once the OPF tail
    // holds at most two systems per compute unit, so that the eigenvalue
    // workgroups fill the CUs that the tail's factorisations leave idle
    // without slowing the full-width launches before it.
    bool go = false;
    if (!dyn_busy && ready > 0) {
      if (ipm_left == 0) go = true;
      else if (eager || (opts.overlap == 1 && assigned >= N)) go = ready >= dyn_min || ipm_left < ready;
      else if (opts.overlap == 2 && assigned >= N) go = ipm_left <= 2 * std::max(c->n_cu, 1);
      else if (assigned < N) go = ready >= dyn_min;
    }
    if (go) {
      const int ndyn = cnt[PH_DYN];
      launch_claim(s, nslots, st);
      HIPCHK(hipEventRecord(ev_ipm, st));
      HIPCHK(hipStreamWaitEvent(sd, ev_ipm, 0));
      rc = timed(CS_K_DYN_ASSEMBLE, sd, ndyn, -1, [&] { launch_dyn_assemble(*D, s, nslots, sd); });
      if (rc != CS_OK) return rc;
      rc = timed(CS_K_DYN_LU, sd, ndyn, -1, [&] {
        launch_lu_solve(s.K, s.k_stride, s.ny, s.nyc, s.ldy, s.piv, pstride, s.st, PH_DYNB, 1,
                        nslots, nullptr, sd, LU_DYN, ndyn);
      });
      if (rc != CS_OK) return rc;
      rc = timed(CS_K_STATE_MATRIX, sd, ndyn, -1, [&] { launch_form_state(*D, s, nslots, sd); });
      if (rc != CS_OK) return rc;
      rc = timed(CS_K_EIG, sd, ndyn, -1, [&] {
        launch_eig(s.A, s.a_stride, s.lda_a, nullptr, 0, s.wr, s.wi, s.na, s.st, nslots,
                   nullptr, s.K, s.k_stride, sd);
      });
      if (rc != CS_OK) return rc;
      rc = timed(CS_K_CLASSIFY, sd, ready, -1, [&] {
        launch_classify(s, nslots, opts.near_eps, opts.max_it, d_res, item_req, req_done,
                        detail, D->nb, D->ng, sd);
      });
      if (rc != CS_OK) return rc;
      HIPCHK(hipEventRecord(ev_dyn, sd));
      if (T) c->stats.dyn_order = s.ny;
      dyn_busy = true;
      return CS_OK;
    }
    const bool can_refill = assigned < N && cnt[PH_EMPTY] > 0;
    if (ipm_left == 0 && !can_refill) {
      if (dyn_busy) {
        // nothing to iterate: wait for the dynamic stage to free its slots
        if (!may_block) {
          *waiting = true;
          return CS_OK;
        }
        HIPCHK(hipEventSynchronize(ev_dyn));
        dyn_busy = false;
        return count();
      }
      if (ready == 0) {
        if (assigned >= N) {
          idle = true;
          return CS_OK;
        }
        return fail(CS_EDEVICE, "scenario slots in an unexpected state");
      }
    }
    return CS_OK;
  }

  // the given stream continues after both of the engine's streams
  int join(hipStream_t after) {
    HIPCHK(hipEventRecord(ev_dyn, sd));
    HIPCHK(hipStreamWaitEvent(after, ev_dyn, 0));
    return CS_OK;
  }
};

// ------------------------------------------------------------------ screen
static int check_opts(const cs_opts& opts, const char* who) {
  if (opts.prec != CS_PREC_FP64 && opts.prec != CS_PREC_MIXED)
    return fail(CS_EINVAL, std::string(who) + ": prec must be CS_PREC_FP64 or CS_PREC_MIXED");
  if (opts.max_it < 1 || opts.max_it > 10000) return fail(CS_EINVAL, std::string(who) + ": max_it out of range");
  if (!(opts.tol > 0)) return fail(CS_EINVAL, std::string(who) + ": tol must be > 0");
  if (opts.refine_steps < 0 || opts.refine_steps > 100)
    return fail(CS_EINVAL, std::string(who) + ": refine_steps must be in 0..100");
  if (opts.graph < 0 || opts.graph > 64)
    return fail(CS_EINVAL, std::string(who) + ": graph must be in 0..64");
  if (opts.autotune != 0 && opts.autotune != 1)
    return fail(CS_EINVAL, std::string(who) + ": autotune must be 0 or 1");
  if (opts.overlap < 0 || opts.overlap > 2)
    return fail(CS_EINVAL, std::string(who) + ": overlap must be 0, 1 or 2");
  return CS_OK;
}

// ------------------------------------------------------------------ autotuning
// Launch variant of the batched LU for order n: every candidate times one
// launch over min(batch, 512) (large orders) or min(batch, 2048) (orders the
// register-resident kernel takes) synthetic systems of order n, after one
// untimed launch; the fastest is kept for (device, n, precision).
// Large orders: the panel code of k_lu_big.  Up to lu_reg_order(): the
// wavefronts per matrix of k_lu_solve (four only up to lu_reg_order_w4()).
static const int kTunePanels[CS_TUNE_VARIANTS] = {16, 32, 64, 1664, 3264};
static const int kTuneWaves[2] = {4, 8};

static int tune_lu(cs_ctx* c, int n, bool f32, int batch, int* choice, double* ms) {
  const bool reg = n <= lu_reg_order();
  const size_t es = f32 ? sizeof(float) : sizeof(double);
  const int ncols = n + 1;
  const int lda = (int)round_up(ncols, 2);
  const size_t stride = (size_t)n * lda;
  long long count = std::max(1, std::min(batch, reg ? 2048 : 512));
  const size_t cap = std::max<size_t>(c->hbm_budget / 2, stride * es);
  count = std::max<long long>(1, std::min<long long>(count, (long long)(cap / (stride * es))));
  void* A = nullptr;
  int* piv = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&] {
    if (A) hipFree(A);
    if (piv) hipFree(piv);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
  };
  if (hipMalloc(&A, stride * es * count) != hipSuccess ||
      hipMalloc(&piv, sizeof(int) * (size_t)n * count) != hipSuccess) {
    cleanup();
    return fail(CS_ENOMEM, "cs_autotune: allocation failed");
  }
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(CS_EDEVICE, "cs_autotune: event creation failed");
  }
  hipStream_t st = c->stream;
  const int nvar = reg ? (n <= lu_reg_order_w4() ? 2 : 1) : CS_TUNE_VARIANTS;
  int best = 0;
  float best_ms = 0.0f;
  for (int v = 0; v < nvar; ++v) {
    // a register-resident order with only eight wavefronts possible times that one
    const int nb = reg ? (nvar == 1 ? 8 : kTuneWaves[v]) : kTunePanels[v];
    if (reg) lu_set_variant(c->device, n, f32, nb);
    float t = 0.0f;
    for (int rep = 0; rep < 2; ++rep) {
      launch_tune_fill(A, f32, stride, n, ncols, lda, (int)count, 12345u + rep, st);
      hipEventRecord(e0, st);
      if (reg && f32)
        launch_lu_solve_f32(static_cast<float*>(A), stride, n, ncols, lda, piv, n, nullptr, 0,
                            0, (int)count, nullptr, st);
      else if (reg)
        launch_lu_solve(static_cast<double*>(A), stride, n, ncols, lda, piv, n, nullptr, 0, 0,
                        (int)count, nullptr, st);
      else if (f32)
        launch_lu_big_f32(static_cast<float*>(A), stride, n, ncols, lda, piv, n, nullptr, 0, 0,
                          (int)count, nullptr, st, nb);
      else
        launch_lu_big(static_cast<double*>(A), stride, n, ncols, lda, piv, n, nullptr, 0, 0,
                      (int)count, nullptr, st, nb);
      hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
        if (reg) lu_set_variant(c->device, n, f32, 0);
        cleanup();
        return fail(CS_EDEVICE, "cs_autotune: timing launch failed");
      }
    }
    if (ms) ms[reg && nvar == 1 ? 1 : v] = t;
    if (v == 0 || t < best_ms) {
      best_ms = t;
      best = nb;
    }
  }
  cleanup();
  HIPCHK(hipGetLastError());
  lu_set_variant(c->device, n, f32, best);
  if (choice) *choice = best;
  return CS_OK;
}

extern "C" int cs_autotune(cs_ctx* c, int32_t n, int32_t prec, int32_t batch, int32_t* choice,
                           double* ms) {
  if (!c || n <= 0 || batch <= 0 || (prec != CS_PREC_FP64 && prec != CS_PREC_MIXED))
    return fail(CS_EINVAL, "cs_autotune: bad arguments");
  if (n > lu_max_order())
    return fail(CS_EUNSUPPORTED, "cs_autotune: order above " + std::to_string(lu_max_order()));
  if (choice) *choice = 0;
  if (ms)
    for (int v = 0; v < CS_TUNE_VARIANTS; ++v) ms[v] = std::nan("");
  HIPCHK(hipSetDevice(c->device));
  return tune_lu(c, n, prec == CS_PREC_MIXED, batch, choice, ms);
}

extern "C" int cs_autotune_set(cs_ctx* c, int32_t n, int32_t prec, int32_t choice) {
  bool ok = choice == 0;
  if (n <= lu_reg_order())
    ok = ok || choice == 8 || (choice == 4 && n <= lu_reg_order_w4());
  else
    ok = ok || choice == 16 || choice == 32 || choice == 64 || choice == 1664 || choice == 3264;
  if (!c || n <= 0 || (prec != CS_PREC_FP64 && prec != CS_PREC_MIXED) || !ok)
    return fail(CS_EINVAL, "cs_autotune_set: bad arguments");
  lu_set_variant(c->device, n, prec == CS_PREC_MIXED, choice);
  return CS_OK;
}

// opts.autotune: tune the LU of the KKT order once per process
static int autotune_for(cs_ctx* c, const Plan& p, const cs_opts& opts, int B) {
  if (!opts.autotune) return CS_OK;
  for (int f = 0; f < 2; ++f) {
    const bool f32 = f == 1;
    if (f32 && opts.prec != CS_PREC_MIXED) continue;
    if (lu_variant(c->device, p.s.nk, f32) != 0) continue;
    const int rc = tune_lu(c, p.s.nk, f32, B, nullptr, nullptr);
    if (rc != CS_OK) return rc;
  }
  return CS_OK;
}

static int run_screen(cs_ctx* c, cs_net* n, const int* d_out_list, long long N,
                      const double* d_lambda, const cs_opts* o, cs_result* d_res,
                      double* d_risk, hipStream_t st, Plan* keep,
                      const DetailOut* detail = nullptr, bool in_scratch = false,
                      int width = 2) {
  cs_opts opts;
  cs_opts_default(&opts);
  if (o) opts = *o;
  int rc = check_opts(opts, "cs_screen");
  if (rc != CS_OK) return rc;
  HIPCHK(hipSetDevice(c->device));
  // an error another runtime call left pending is not this call's
  (void)hipGetLastError();
  Plan p = plan_sizes(n, opts.prec == CS_PREC_MIXED);
  const size_t budget = opts.hbm_budget ? opts.hbm_budget : c->hbm_budget;
  if (p.per_slot > budget)
    return fail(CS_EHBM, "cs_screen: one scenario needs " + std::to_string(p.per_slot) +
                             " bytes, over the budget of " + std::to_string(budget));
  long long B = (long long)(budget / p.per_slot);
  if (opts.batch > 0) B = std::min<long long>(B, opts.batch);
  B = std::max<long long>(1, std::min<long long>(B, std::max<long long>(N, 1)));
  B = std::min<long long>(B, 1 << 20);
  if (in_scratch) {
    // as many slots as the static scratch holds (the layout pads each array)
    if (p.per_slot > CS_NOALLOC_SCRATCH_BYTES / 2)
      return fail(CS_EHBM, "cs_screen_device_noalloc: one scenario needs " +
                               std::to_string(p.per_slot) + " bytes of workspace, above half the " +
                               std::to_string((size_t)CS_NOALLOC_SCRATCH_BYTES) +
                               "-byte static scratch");
    B = std::min<long long>(B, (long long)(CS_NOALLOC_SCRATCH_BYTES / p.per_slot) - 1);
    while (B > 1 && bind_workspace(nullptr, nullptr, n, p, (int)B, c->scratch,
                                   CS_NOALLOC_SCRATCH_BYTES) != CS_OK)
      B = B * 15 / 16;
    rc = bind_workspace(nullptr, nullptr, n, p, (int)B, c->scratch, CS_NOALLOC_SCRATCH_BYTES);
  } else {
    rc = bind_workspace(&c->ws, &c->ws_bytes, n, p, (int)B);
  }
  if (rc != CS_OK) return rc;
  const bool tm = opts.timing != 0;
  if (tm && c->units_cap == 0) {
    const size_t cap = 1 << 20;
    HIPCHK(hipMalloc(&c->d_units, sizeof(int) * cap));
    c->units_cap = cap;
  }
  if ((rc = autotune_for(c, p, opts, (int)B)) != CS_OK) return rc;
  TimedLaunches T(c, tm);
  Engine e;
  e.c = c;
  e.D = &n->d;
  e.s = p.s;
  e.opts = opts;
  e.nslots = (int)B;
  e.pstride = std::max(p.s.nk, p.s.ny);
  e.dyn_min = std::max(1, std::min((int)B, 1024));
  e.st = st;
  e.sd = opts.overlap ? c->stream_dyn : st;
  e.ev_ipm = c->ev_ipm;
  e.ev_dyn = c->ev_dyn;
  e.d_next = reinterpret_cast<unsigned long long*>(c->d_sched);
  e.d_counts = c->d_sched + 2;
  e.h_counts = c->h_sched + 2;
  e.h_next = reinterpret_cast<unsigned long long*>(c->h_sched);
  e.d_list = d_out_list;
  e.d_res = d_res;
  e.q_cap = std::max<long long>(N, 1);
  e.T = tm ? &T : nullptr;
  e.detail = detail;
  e.width = width;
  c->stats.kkt_order = p.s.nk;
  if ((rc = e.start()) != CS_OK) return rc;
  // every scenario needs at most max_it + 2 rounds in its slot, plus a few
  // rounds per dynamic stage; a loop beyond this bound is an internal error
  const long long max_rounds = ((N + B - 1) / B + 2) * (long long)(opts.max_it + 8) * 4 + 1000;
  long long rounds = 0;
  for (;;) {
    bool idle = false;
    if ((rc = e.round(N, idle)) != CS_OK) return rc;
    if (idle) break;
    if (++rounds > max_rounds) return fail(CS_EDEVICE, "cs_screen: scheduling did not finish");
  }
  if ((rc = e.join(st)) != CS_OK) return rc;
  HIPCHK(hipGetLastError());
  if (d_risk) {
    const int n_comp = n->nl + n->ng + n->nd;
    rc = T.run(CS_K_RISK, st, n_comp, -1, [&] {
      launch_risk(d_out_list, N, reinterpret_cast<const uint8_t*>(d_res), (int)sizeof(cs_result),
                  d_lambda, n_comp, d_risk, st, width);
    });
    if (rc != CS_OK) return rc;
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  if ((rc = T.resolve()) != CS_OK) return rc;
  if (keep) *keep = p;
  return CS_OK;
}

static int validate_host(const cs_net* n, const int32_t* outages, int64_t N, const double* lam) {
  const int n_comp = n->nl + n->ng + n->nd;
  for (int64_t i = 0; i < N; ++i) {
    const int a = outages[2 * i], b = outages[2 * i + 1];
    if (a == -1 && b == -1) continue;   // the base case: nothing out
    if (a < 0 || a >= n_comp)
      return fail(CS_EINVAL, "outage row " + std::to_string(i) + ": component id out of range");
    if (b != -1 && (b < 0 || b >= n_comp || b == a))
      return fail(CS_EINVAL, "outage row " + std::to_string(i) +
                                 ": second id must be -1 or a distinct valid id");
  }
  if (lam)
    for (int i = 0; i < n_comp; ++i)
      if (!(lam[i] >= 0) || !std::isfinite(lam[i]))
        return fail(CS_EINVAL, "failure rate " + std::to_string(i) + " must be finite and >= 0");
  return CS_OK;
}

extern "C" int cs_screen(cs_ctx* c, cs_net* n, const int32_t* outages, int64_t N,
                         const double* lambda, const cs_opts* opts, cs_result* out,
                         double* risk) {
  if (!c || !n || (N > 0 && (!outages || !out)) || N < 0)
    return fail(CS_EINVAL, "cs_screen: NULL argument or negative n");
  if (risk && !lambda) return fail(CS_EINVAL, "cs_screen: risk requested without lambda");
  int rc = validate_host(n, outages, N, lambda);
  if (rc != CS_OK) return rc;
  const int n_comp = n->nl + n->ng + n->nd;
  if (N == 0) {
    if (risk)
      for (int i = 0; i < n_comp; ++i) risk[i] = 0.0;
    return CS_OK;
  }
  HIPCHK(hipSetDevice(c->device));
  int* d_list = nullptr;
  double* d_lam = nullptr;
  cs_result* d_res = nullptr;
  double* d_risk = nullptr;
  auto cleanup = [&]() {
    if (d_list) hipFree(d_list);
    if (d_lam) hipFree(d_lam);
    if (d_res) hipFree(d_res);
    if (d_risk) hipFree(d_risk);
  };
  if (hipMalloc(&d_list, sizeof(int) * 2 * N) != hipSuccess ||
      hipMalloc(&d_res, sizeof(cs_result) * N) != hipSuccess ||
      (risk && (hipMalloc(&d_lam, sizeof(double) * n_comp) != hipSuccess ||
                hipMalloc(&d_risk, sizeof(double) * n_comp) != hipSuccess))) {
    cleanup();
    return fail(CS_ENOMEM, "cs_screen: device allocation failed");
  }
  if (hipMemcpy(d_list, outages, sizeof(int) * 2 * N, hipMemcpyHostToDevice) != hipSuccess ||
      (risk && hipMemcpy(d_lam, lambda, sizeof(double) * n_comp, hipMemcpyHostToDevice) != hipSuccess)) {
    cleanup();
    return fail(CS_EDEVICE, "cs_screen: copy to device failed");
  }
  rc = run_screen(c, n, d_list, N, d_lam, opts, d_res, d_risk, c->stream, nullptr);
  if (rc == CS_OK) {
    if (hipMemcpy(out, d_res, sizeof(cs_result) * N, hipMemcpyDeviceToHost) != hipSuccess ||
        (risk && hipMemcpy(risk, d_risk, sizeof(double) * n_comp, hipMemcpyDeviceToHost) != hipSuccess))
      rc = fail(CS_EDEVICE, "cs_screen: copy to host failed");
  }
  cleanup();
  return rc;
}

static int screen_device(const char* who, cs_ctx* c, cs_net* n, const int32_t* d_outages,
                         int64_t N, const double* d_lambda, const cs_opts* opts,
                         cs_result* d_out, double* d_risk, void* stream, bool in_scratch,
                         int width = 2) {
  if (!c || !n || N < 0 || (N > 0 && (!d_outages || !d_out)))
    return fail(CS_EINVAL, std::string(who) + ": NULL argument or negative n");
  if (d_risk && !d_lambda) return fail(CS_EINVAL, std::string(who) + ": risk requested without lambda");
  if (in_scratch && opts && opts->timing)
    return fail(CS_EINVAL, std::string(who) + ": kernel timing is not available (it allocates)");
  if (in_scratch && opts && (opts->graph || opts->autotune))
    return fail(CS_EINVAL, std::string(who) + ": graphs and autotuning are not available (they allocate)");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = stream ? static_cast<hipStream_t>(stream) : c->stream;
  const int n_comp = n->nl + n->ng + n->nd;
  // validate the list (bit 1) and the rates (bit 2) on the device
  HIPCHK(hipMemsetAsync(c->d_counter, 0, sizeof(int), st));
  launch_validate(d_outages, N, n_comp, c->d_counter, st, width);
  if (d_lambda) launch_validate_rates(d_lambda, n_comp, c->d_counter, st);
  HIPCHK(hipMemcpyAsync(c->h_counter, c->d_counter, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (*c->h_counter & 1) return fail(CS_EINVAL, std::string(who) + ": invalid outage row in the list");
  if (*c->h_counter & 2)
    return fail(CS_EINVAL, std::string(who) + ": every failure rate must be finite and >= 0");
  if (N == 0) {
    if (d_risk) HIPCHK(hipMemsetAsync(d_risk, 0, sizeof(double) * n_comp, st));
    HIPCHK(hipStreamSynchronize(st));
    return CS_OK;
  }
  return run_screen(c, n, d_outages, N, d_lambda, opts, d_out, d_risk, st, nullptr, nullptr,
                    in_scratch, width);
}

extern "C" int cs_screen_device(cs_ctx* c, cs_net* n, const int32_t* d_outages, int64_t N,
                                const double* d_lambda, const cs_opts* opts, cs_result* d_out,
                                double* d_risk, void* stream) {
  return screen_device("cs_screen_device", c, n, d_outages, N, d_lambda, opts, d_out, d_risk,
                       stream, false);
}

extern "C" int cs_screen_device_noalloc(cs_ctx* c, cs_net* n, const int32_t* d_outages,
                                        int64_t N, const double* d_lambda, const cs_opts* opts,
                                        cs_result* d_out, double* d_risk, void* stream) {
  return screen_device("cs_screen_device_noalloc", c, n, d_outages, N, d_lambda, opts, d_out,
                       d_risk, stream, true);
}

// ------------------------------------------------------------------ serving
// A server runs one lane per network: the lane's scenario slots (its part of
// the HBM budget), its device ring of outage pairs and records, its streams
// and its engine.  One host thread drives every lane: it issues a round on
// each lane that has work (their launches overlap on the device, each lane
// on its own streams), then settles them in turn, then finishes the requests
// whose records are all in.
struct cs_req {
  cs_server* srv = nullptr;
  int lane = 0;                          // network index
  int slot = -1;                         // request table index
  long long q0 = 0;                      // first ring position (absolute)
  int64_t n = 0;
  int n_comp = 0;
  bool has_lam = false;
  std::vector<double> lam;
  std::vector<cs_result> res;
  std::vector<double> risk;
  bool done = false, freed = false;
  int status = CS_OK;
  std::string msg;
  std::chrono::steady_clock::time_point t0, t1;
};

struct ServerLane {
  cs_net* n = nullptr;
  Plan p;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t st = nullptr, sd = nullptr;
  hipEvent_t ev_ipm = nullptr, ev_dyn = nullptr;
  int* q_out = nullptr;                  // ring of outage pairs
  cs_result* q_res = nullptr;            // ring of records
  int* item_req = nullptr;               // ring: request table index per scenario
  double* req_scale = nullptr;           // [R][n_load] each request's load factors
  int* d_sched = nullptr;                // next (64-bit) + stage counts
  int* h_sched = nullptr;
  int* g_out = nullptr;                  // one request's list, contiguous
  cs_result* g_res = nullptr;
  double* g_lam = nullptr;
  double* g_risk = nullptr;
  long long submitted = 0;               // scenarios admitted (absolute)
  long long seen = 0;                    // scenarios the engine has been told about
  bool idle = false;                     // every admitted scenario recorded
  bool waiting = false;                  // only the dynamic stage is left to wait for
  bool pending = false;                  // a round issued and not yet settled
  long long n_issued = 0;                // scenarios available when it was issued
  hipEvent_t ev_round = nullptr;         // recorded after the round's stage counts
  Engine e;
};

struct cs_server {
  static constexpr int R = 1024;         // requests in flight at most
  cs_ctx* c = nullptr;
  int device = 0;
  cs_opts opts{};
  long long q_cap = 0;                   // ring capacity per lane
  std::vector<ServerLane*> lanes;
  int* req_done = nullptr;               // [R] records completed per request
  int* h_req_done = nullptr;             // pinned copy
  hipStream_t scopy = nullptr;
  std::vector<cs_req*> table;            // requests in flight
  std::set<cs_req*> owned;               // every request not yet freed by the caller
  std::mutex m;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  int error = CS_OK;
  std::string error_msg;
  std::thread th;
};

// Finish every request whose records are all in: gather its slice of its
// lane's ring, reduce its R_i, copy to the host.  The gather runs on the
// stream of the lane's dynamic stage (e.sd), after the records it reads.
static int server_complete(cs_server* S) {
  std::vector<cs_req*> live;
  {
    std::lock_guard<std::mutex> lk(S->m);
    for (cs_req* r : S->table)
      if (r && !r->done) live.push_back(r);
  }
  if (live.empty()) return CS_OK;
  HIPCHK(hipMemcpyAsync(S->h_req_done, S->req_done, sizeof(int) * cs_server::R,
                        hipMemcpyDeviceToHost, S->scopy));
  HIPCHK(hipStreamSynchronize(S->scopy));
  for (cs_req* r : live) {
    if (S->h_req_done[r->slot] < r->n) continue;
    ServerLane& L = *S->lanes[r->lane];
    launch_gather_request(L.q_out, L.q_res, r->q0, (int)r->n, S->q_cap, L.g_out, L.g_res, L.e.sd);
    if (r->has_lam) {
      HIPCHK(hipMemcpyAsync(L.g_lam, r->lam.data(), sizeof(double) * r->n_comp,
                            hipMemcpyHostToDevice, L.e.sd));
      launch_risk(L.g_out, r->n, reinterpret_cast<const uint8_t*>(L.g_res),
                  (int)sizeof(cs_result), L.g_lam, r->n_comp, L.g_risk, L.e.sd);
      r->risk.resize(r->n_comp);
      HIPCHK(hipMemcpyAsync(r->risk.data(), L.g_risk, sizeof(double) * r->n_comp,
                            hipMemcpyDeviceToHost, L.e.sd));
    }
    r->res.resize(r->n);
    HIPCHK(hipMemcpyAsync(r->res.data(), L.g_res, sizeof(cs_result) * r->n,
                          hipMemcpyDeviceToHost, L.e.sd));
    HIPCHK(hipStreamSynchronize(L.e.sd));
    std::lock_guard<std::mutex> lk(S->m);
    r->t1 = std::chrono::steady_clock::now();
    r->done = true;
    S->table[r->slot] = nullptr;
    if (r->freed) {
      S->owned.erase(r);
      delete r;
    }
  }
  S->cv_done.notify_all();
  return CS_OK;
}

static void server_fail_all(cs_server* S, int code, const std::string& msg) {
  std::lock_guard<std::mutex> lk(S->m);
  S->error = code;
  S->error_msg = msg;
  for (cs_req*& r : S->table) {
    if (!r) continue;
    r->status = code;
    r->msg = msg;
    r->done = true;
    r->t1 = std::chrono::steady_clock::now();
    if (r->freed) {
      S->owned.erase(r);
      delete r;
    }
    r = nullptr;
  }
  S->cv_done.notify_all();
}

// One network: each round is issued and settled in turn, and the engine may
// block on its own dynamic stage.
static void server_loop_one(cs_server* S) {
  ServerLane& L = *S->lanes[0];
  int rc = CS_OK;
  for (;;) {
    long long N;
    {
      std::lock_guard<std::mutex> lk(S->m);
      N = L.submitted;
    }
    bool idle = false;
    if ((rc = L.e.round(N, idle)) != CS_OK || (rc = server_complete(S)) != CS_OK) {
      server_fail_all(S, rc, g_err);
      return;
    }
    if (idle) {
      std::unique_lock<std::mutex> lk(S->m);
      S->cv_work.wait(lk, [&] { return S->stop || L.submitted > N; });
      if (S->stop && L.submitted == N) return;
    }
  }
}

// Several networks: every lane advances at its own pace.  A lane's round is
// issued, an event marks the end of its stage counts, and the round is
// settled when that event has completed, so that a lane with short rounds
// (a small network) is never held to the pace of one with long rounds.
// With nothing to settle or issue the thread sleeps for a few microseconds.
static void server_loop_many(cs_server* S) {
  const size_t nl = S->lanes.size();
  int rc = CS_OK;
  std::vector<long long> N(nl);
  for (;;) {
    {
      std::lock_guard<std::mutex> lk(S->m);
      for (size_t i = 0; i < nl; ++i) N[i] = S->lanes[i]->submitted;
    }
    bool progress = false;
    for (size_t i = 0; i < nl && rc == CS_OK; ++i) {
      ServerLane& L = *S->lanes[i];
      if (!L.pending) {
        if (L.idle && N[i] <= L.seen) continue;
        if (L.waiting && !L.idle) {
          // only the dynamic stage is left: issue again once it has ended
          const hipError_t q = hipEventQuery(L.e.ev_dyn);
          if (q == hipErrorNotReady) continue;
          if (q != hipSuccess) {
            rc = fail(CS_EDEVICE, "dynamic stage failed");
            break;
          }
        }
        if ((rc = L.e.issue(N[i])) != CS_OK) break;
        if (hipEventRecord(L.ev_round, L.st) != hipSuccess) {
          rc = fail(CS_EDEVICE, "server: event record failed");
          break;
        }
        L.n_issued = N[i];
        L.pending = true;
        progress = true;
      } else {
        const hipError_t q = hipEventQuery(L.ev_round);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) {
          rc = fail(CS_EDEVICE, "server: round failed");
          break;
        }
        bool idle = false, waiting = false;
        if ((rc = L.e.settle(L.n_issued, idle, false, &waiting)) != CS_OK) break;
        L.idle = idle;
        L.waiting = waiting;
        L.seen = L.n_issued;
        L.pending = false;
        progress = true;
      }
    }
    if (rc != CS_OK || (rc = server_complete(S)) != CS_OK) {
      server_fail_all(S, rc, g_err);
      return;
    }
    bool all_idle = true;
    for (ServerLane* L : S->lanes) all_idle = all_idle && L->idle && !L->pending;
    if (all_idle) {
      std::unique_lock<std::mutex> lk(S->m);
      S->cv_work.wait(lk, [&] {
        if (S->stop) return true;
        for (size_t i = 0; i < nl; ++i)
          if (S->lanes[i]->submitted > N[i]) return true;
        return false;
      });
      if (S->stop) {
        bool more = false;
        for (size_t i = 0; i < nl; ++i) more = more || S->lanes[i]->submitted > N[i];
        if (!more) return;
      }
    } else if (!progress) {
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }
}

static void server_loop(cs_server* S) {
  hipSetDevice(S->device);
  for (ServerLane* L : S->lanes) {
    const int rc = L->e.start();
    if (rc != CS_OK) {
      server_fail_all(S, rc, g_err);
      return;
    }
  }
  if (S->lanes.size() == 1) server_loop_one(S);
  else server_loop_many(S);
}

static void lane_free(ServerLane* L) {
  for (void* q : {(void*)L->q_out, (void*)L->q_res, (void*)L->item_req, (void*)L->req_scale,
                  (void*)L->d_sched, (void*)L->g_out, (void*)L->g_res, (void*)L->g_lam,
                  (void*)L->g_risk, L->ws})
    if (q) hipFree(q);
  if (L->h_sched) hipHostFree(L->h_sched);
  for (hipStream_t q : {L->st, L->sd})
    if (q) hipStreamDestroy(q);
  for (hipEvent_t q : {L->ev_ipm, L->ev_dyn, L->ev_round})
    if (q) hipEventDestroy(q);
  delete L;
}

// Slots, ring and engine of one lane; bytes is the lane's part of the budget.
static int lane_create(cs_server* S, cs_net* n, size_t bytes, int index, ServerLane** out) {
  const cs_opts& opts = S->opts;
  ServerLane* L = new ServerLane();
  *out = L;
  L->n = n;
  L->p = plan_sizes(n, opts.prec == CS_PREC_MIXED);
  if (L->p.per_slot > bytes)
    return fail(CS_EHBM, "cs_server_create: network " + std::to_string(index) +
                             ": one scenario needs " + std::to_string(L->p.per_slot) +
                             " bytes, over its part of the budget, " + std::to_string(bytes));
  long long B = (long long)(bytes / L->p.per_slot);
  if (opts.batch > 0) B = std::min<long long>(B, opts.batch);
  B = std::max<long long>(1, std::min<long long>(B, 1 << 20));
  int rc = bind_workspace(&L->ws, &L->ws_bytes, n, L->p, (int)B);
  if (rc != CS_OK) return rc;
  if ((rc = autotune_for(S->c, L->p, opts, (int)B)) != CS_OK) return rc;
  const long long qc = S->q_cap;
  const int n_comp = n->nl + n->ng + n->nd;
  if (hipStreamCreateWithFlags(&L->st, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&L->sd, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&L->ev_ipm, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&L->ev_dyn, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&L->ev_round, hipEventDisableTiming) != hipSuccess ||
      hipMalloc(&L->q_out, sizeof(int) * 2 * qc) != hipSuccess ||
      hipMalloc(&L->q_res, sizeof(cs_result) * qc) != hipSuccess ||
      hipMalloc(&L->item_req, sizeof(int) * qc) != hipSuccess ||
      hipMalloc(&L->req_scale, sizeof(double) * (size_t)cs_server::R * std::max(n->nd, 1)) != hipSuccess ||
      hipMalloc(&L->d_sched, sizeof(int) * (PH_COUNT + 3)) != hipSuccess ||
      hipHostMalloc(&L->h_sched, sizeof(int) * (PH_COUNT + 3), hipHostMallocDefault) != hipSuccess ||
      hipMalloc(&L->g_out, sizeof(int) * 2 * qc) != hipSuccess ||
      hipMalloc(&L->g_res, sizeof(cs_result) * qc) != hipSuccess ||
      hipMalloc(&L->g_lam, sizeof(double) * std::max(n_comp, 1)) != hipSuccess ||
      hipMalloc(&L->g_risk, sizeof(double) * std::max(n_comp, 1)) != hipSuccess)
    return fail(CS_ENOMEM, "cs_server_create: allocation failed");
  Engine& e = L->e;
  e.c = S->c;
  e.D = &n->d;
  e.s = L->p.s;
  e.opts = opts;
  e.nslots = (int)B;
  e.pstride = std::max(L->p.s.nk, L->p.s.ny);
  e.dyn_min = std::max(1, std::min((int)B, 1024));
  e.eager = true;
  e.st = L->st;
  // the records a request gathers are written on e.sd (== st without overlap)
  e.sd = opts.overlap ? L->sd : L->st;
  e.ev_ipm = L->ev_ipm;
  e.ev_dyn = L->ev_dyn;
  e.d_next = reinterpret_cast<unsigned long long*>(L->d_sched);
  e.d_counts = L->d_sched + 2;
  e.h_counts = L->h_sched + 2;
  e.h_next = reinterpret_cast<unsigned long long*>(L->h_sched);
  e.d_list = L->q_out;
  e.d_res = L->q_res;
  e.q_cap = qc;
  e.item_req = L->item_req;
  e.load_scale = L->req_scale;
  e.req_done = S->req_done;
  e.T = nullptr;
  return CS_OK;
}

extern "C" int cs_server_create_multi(cs_ctx* c, cs_net* const* nets, int n_nets,
                                      const double* shares, const cs_opts* o,
                                      int64_t queue_capacity, cs_server** out) {
  if (!c || !nets || !out || n_nets < 1 || n_nets > CS_SERVER_MAX_NETS || queue_capacity <= 0 ||
      queue_capacity > (1ll << 30))
    return fail(CS_EINVAL, "cs_server_create: bad arguments");
  *out = nullptr;
  double share_sum = 0.0;
  for (int i = 0; i < n_nets; ++i) {
    if (!nets[i]) return fail(CS_EINVAL, "cs_server_create: NULL network");
    if (nets[i]->device != c->device)
      return fail(CS_EINVAL, "cs_server_create: network made on another device");
    if (shares && !(shares[i] > 0 && std::isfinite(shares[i])))
      return fail(CS_EINVAL, "cs_server_create: shares must be finite and > 0");
    share_sum += shares ? shares[i] : 1.0;
  }
  cs_opts opts;
  cs_opts_default(&opts);
  if (o) opts = *o;
  opts.timing = 0;
  int rc = check_opts(opts, "cs_server_create");
  if (rc != CS_OK) return rc;
  HIPCHK(hipSetDevice(c->device));
  cs_server* S = new cs_server();
  S->c = c;
  S->device = c->device;
  S->opts = opts;
  S->q_cap = queue_capacity;
  S->table.assign(cs_server::R, nullptr);
  const size_t budget = opts.hbm_budget ? opts.hbm_budget : c->hbm_budget;
  auto bail = [&](int code) {
    const std::string msg = g_err;
    cs_server_destroy(S);
    return fail(code, msg);
  };
  if (hipStreamCreateWithFlags(&S->scopy, hipStreamNonBlocking) != hipSuccess ||
      hipMalloc(&S->req_done, sizeof(int) * cs_server::R) != hipSuccess ||
      hipHostMalloc(&S->h_req_done, sizeof(int) * cs_server::R, hipHostMallocDefault) != hipSuccess) {
    fail(CS_ENOMEM, "cs_server_create: allocation failed");
    return bail(CS_ENOMEM);
  }
  if (hipMemset(S->req_done, 0, sizeof(int) * cs_server::R) != hipSuccess) {
    fail(CS_EDEVICE, "cs_server_create: device error");
    return bail(CS_EDEVICE);
  }
  for (int i = 0; i < n_nets; ++i) {
    const double f = (shares ? shares[i] : 1.0) / share_sum;
    ServerLane* L = nullptr;
    rc = lane_create(S, nets[i], (size_t)((double)budget * f), i, &L);
    S->lanes.push_back(L);
    if (rc != CS_OK) return bail(rc);
  }
  S->th = std::thread(server_loop, S);
  *out = S;
  return CS_OK;
}

extern "C" int cs_server_create(cs_ctx* c, cs_net* n, const cs_opts* o,
                                int64_t queue_capacity, cs_server** out) {
  if (!n) return fail(CS_EINVAL, "cs_server_create: bad arguments");
  return cs_server_create_multi(c, &n, 1, nullptr, o, queue_capacity, out);
}

extern "C" int cs_server_slots(const cs_server* S, int net) {
  if (!S || net < 0 || net >= (int)S->lanes.size())
    return fail(CS_EINVAL, "cs_server_slots: bad arguments");
  return S->lanes[net]->e.nslots;
}

extern "C" void cs_server_destroy(cs_server* S) {
  if (!S) return;
  if (S->th.joinable()) {
    {
      std::lock_guard<std::mutex> lk(S->m);
      S->stop = true;
    }
    S->cv_work.notify_all();
    S->th.join();
  }
  hipSetDevice(S->device);
  // requests the caller still holds outlive the server, detached from it
  for (cs_req* r : S->owned) {
    if (r->freed) {
      delete r;
      continue;
    }
    if (!r->done) {
      r->status = CS_EDEVICE;
      r->msg = "server destroyed";
      r->done = true;
    }
    r->srv = nullptr;
  }
  for (ServerLane* L : S->lanes)
    if (L) lane_free(L);
  if (S->req_done) hipFree(S->req_done);
  if (S->h_req_done) hipHostFree(S->h_req_done);
  if (S->scopy) hipStreamDestroy(S->scopy);
  delete S;
}

extern "C" int cs_submit_net(cs_server* S, int net, const int32_t* outages, int64_t n,
                             const double* lambda, const double* load_scale, cs_req** out) {
  if (!S || !out || n < 0 || (n > 0 && !outages)) return fail(CS_EINVAL, "cs_submit: bad arguments");
  *out = nullptr;
  if (net < 0 || net >= (int)S->lanes.size())
    return fail(CS_EINVAL, "cs_submit: network index " + std::to_string(net) + " out of range");
  if (n > S->q_cap) return fail(CS_EINVAL, "cs_submit: request longer than the ring");
  ServerLane& L = *S->lanes[net];
  int rc = validate_host(L.n, outages, n, lambda);
  if (rc != CS_OK) return rc;
  const int n_comp = L.n->nl + L.n->ng + L.n->nd;
  const int nd = L.n->nd;
  std::vector<double> scale(std::max(nd, 1), 1.0);
  if (load_scale) {
    for (int d = 0; d < nd; ++d) {
      if (!(load_scale[d] >= 0) || !std::isfinite(load_scale[d]))
        return fail(CS_EINVAL, "cs_submit_snapshot: load factor " + std::to_string(d) +
                                   " must be finite and >= 0");
      scale[d] = load_scale[d];
    }
  }
  std::unique_lock<std::mutex> lk(S->m);
  if (S->error != CS_OK) return fail(S->error, "cs_submit: server failed: " + S->error_msg);
  long long oldest = L.submitted;
  int slot = -1;
  for (int i = 0; i < cs_server::R; ++i) {
    const cs_req* r = S->table[i];
    if (r && r->lane == net) oldest = std::min(oldest, r->q0);
    else if (!r && slot < 0) slot = i;
  }
  if (slot < 0 || L.submitted + n - oldest > S->q_cap)
    return fail(CS_EAGAIN, "cs_submit: no room for the request right now");
  cs_req* r = new cs_req();
  r->srv = S;
  r->lane = net;
  r->slot = slot;
  r->q0 = L.submitted;
  r->n = n;
  r->n_comp = n_comp;
  r->has_lam = lambda != nullptr;
  if (lambda) r->lam.assign(lambda, lambda + n_comp);
  r->t0 = std::chrono::steady_clock::now();
  S->owned.insert(r);
  if (n == 0) {
    r->done = true;
    r->t1 = r->t0;
    if (lambda) r->risk.assign(n_comp, 0.0);
    *out = r;
    return CS_OK;
  }
  hipSetDevice(S->device);
  // copy into the ring (in two pieces when it wraps), tag the request
  const long long p0 = r->q0 % S->q_cap;
  const long long first = std::min<long long>(n, S->q_cap - p0);
  bool ok = hipMemcpyAsync(L.q_out + 2 * p0, outages, sizeof(int) * 2 * first,
                           hipMemcpyHostToDevice, S->scopy) == hipSuccess;
  if (ok && first < n)
    ok = hipMemcpyAsync(L.q_out, outages + 2 * first, sizeof(int) * 2 * (n - first),
                        hipMemcpyHostToDevice, S->scopy) == hipSuccess;
  if (ok && nd > 0)
    ok = hipMemcpyAsync(L.req_scale + (size_t)slot * nd, scale.data(), sizeof(double) * nd,
                        hipMemcpyHostToDevice, S->scopy) == hipSuccess;
  if (ok) {
    launch_fill_req(L.item_req, r->q0, (int)n, S->q_cap, slot, S->scopy);
    ok = hipMemsetAsync(S->req_done + slot, 0, sizeof(int), S->scopy) == hipSuccess &&
         hipStreamSynchronize(S->scopy) == hipSuccess;
  }
  if (!ok) {
    S->owned.erase(r);
    delete r;
    return fail(CS_EDEVICE, "cs_submit: copy to the device failed");
  }
  S->table[slot] = r;
  L.submitted += n;
  lk.unlock();
  S->cv_work.notify_all();
  *out = r;
  return CS_OK;
}

extern "C" int cs_submit(cs_server* S, const int32_t* outages, int64_t n, const double* lambda,
                         cs_req** out) {
  return cs_submit_net(S, 0, outages, n, lambda, nullptr, out);
}

extern "C" int cs_submit_snapshot(cs_server* S, const int32_t* outages, int64_t n,
                                  const double* lambda, const double* load_scale,
                                  cs_req** out) {
  return cs_submit_net(S, 0, outages, n, lambda, load_scale, out);
}

extern "C" int cs_wait(cs_req* r, int64_t timeout_us, cs_result* out, double* risk,
                       double* latency_s) {
  if (!r) return fail(CS_EINVAL, "cs_wait: NULL request");
  cs_server* S = r->srv;
  if (S) {
    std::unique_lock<std::mutex> lk(S->m);
    auto ready = [&] { return r->done; };
    if (timeout_us < 0) S->cv_done.wait(lk, ready);
    else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
      return fail(CS_ETIMEDOUT, "cs_wait: request not complete");
  }
  if (!r->done) return fail(CS_ETIMEDOUT, "cs_wait: request not complete");
  if (r->status != CS_OK) return fail(r->status, "cs_wait: " + r->msg);
  if (out && r->n) std::memcpy(out, r->res.data(), sizeof(cs_result) * r->n);
  if (risk && r->has_lam) std::memcpy(risk, r->risk.data(), sizeof(double) * r->risk.size());
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t1 - r->t0).count();
  return CS_OK;
}

extern "C" void cs_req_free(cs_req* r) {
  if (!r) return;
  cs_server* S = r->srv;
  if (!S) {
    delete r;
    return;
  }
  std::lock_guard<std::mutex> lk(S->m);
  if (r->done) {
    S->owned.erase(r);
    delete r;
  } else {
    r->freed = true;
  }
}

extern "C" int cs_detail(cs_ctx* c, cs_net* n, const int32_t outage[2], const cs_opts* opts,
                         cs_result* rec, double* vm, double* va, double* pg, double* qg,
                         double* eig_re, double* eig_im, int32_t* n_eig, int32_t* label) {
  if (!c || !n || !outage || !rec) return fail(CS_EINVAL, "cs_detail: NULL argument");
  int rc = validate_host(n, outage, 1, nullptr);
  if (rc != CS_OK) return rc;
  HIPCHK(hipSetDevice(c->device));
  int* d_list = nullptr;
  cs_result* d_res = nullptr;
  if (hipMalloc(&d_list, sizeof(int) * 2) != hipSuccess ||
      hipMalloc(&d_res, sizeof(cs_result)) != hipSuccess) {
    if (d_list) hipFree(d_list);
    return fail(CS_ENOMEM, "cs_detail: allocation failed");
  }
  cs_opts o;
  cs_opts_default(&o);
  if (opts) o = *opts;
  o.batch = 1;
  Plan p;
  hipMemcpy(d_list, outage, sizeof(int) * 2, hipMemcpyHostToDevice);
  rc = run_screen(c, n, d_list, 1, nullptr, &o, d_res, nullptr, c->stream, &p);
  if (rc == CS_OK) {
    const Slots& s = p.s;
    const int nb = n->nb, ng = n->ng;
    std::vector<double> x(s.nx), wr(std::max(s.na, 1)), wi(std::max(s.na, 1));
    std::vector<uint8_t> bus_on(nb), gen_on(ng);
    std::vector<int> lab(nb);
    SlotState S;
    bool ok = hipMemcpy(rec, d_res, sizeof(cs_result), hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(x.data(), s.x, sizeof(double) * s.nx, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(wr.data(), s.wr, sizeof(double) * s.na, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(wi.data(), s.wi, sizeof(double) * s.na, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(bus_on.data(), s.bus_on, nb, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(gen_on.data(), s.gen_on, ng, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(lab.data(), s.label, sizeof(int) * nb, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(&S, s.st, sizeof(SlotState), hipMemcpyDeviceToHost) == hipSuccess;
    if (!ok) {
      rc = fail(CS_EDEVICE, "cs_detail: copy to host failed");
    } else {
      const double nan = std::nan("");
      const bool solved = rec->opf_status != CS_OPF_NOT_RUN;
      for (int b = 0; b < nb; ++b) {
        const bool on = solved && bus_on[b];
        if (va) va[b] = on ? x[b] : nan;
        if (vm) vm[b] = on ? x[nb + b] : nan;
        if (label) label[b] = lab[b];
      }
      for (int g = 0; g < ng; ++g) {
        const bool on = solved && gen_on[g];
        if (pg) pg[g] = on ? x[2 * nb + g] : nan;
        if (qg) qg[g] = on ? x[2 * nb + ng + g] : nan;
      }
      const int ne = (rec->opf_status == CS_OPF_CONVERGED && S.qr_fail == 0) ? rec->n_states : 0;
      if (n_eig) *n_eig = ne;
      for (int i = 0; i < ne; ++i) {
        if (eig_re) eig_re[i] = wr[i];
        if (eig_im) eig_im[i] = wi[i];
      }
    }
  }
  hipFree(d_list);
  hipFree(d_res);
  return rc;
}

extern "C" int cs_dense_solve_batched(const cs_ctx* c, double* d_A, int32_t n, int32_t nrhs,
                                      int32_t lda, int32_t batch, int32_t* d_info, void* stream) {
  if (!c || !d_A || n <= 0 || nrhs < 0 || lda < n + nrhs || batch < 0)
    return fail(CS_EINVAL, "cs_dense_solve_batched: bad arguments");
  if (n > lu_max_order())
    return fail(CS_EUNSUPPORTED, "cs_dense_solve_batched: n = " + std::to_string(n) +
                                     " above the largest supported order " +
                                     std::to_string(lu_max_order()));
  if (lu_lds_bytes(n, nrhs) > c->lds_max)
    return fail(CS_EUNSUPPORTED, "cs_dense_solve_batched: n = " + std::to_string(n) +
                                     " needs more LDS than the device allows (" +
                                     std::to_string(c->lds_max) + " bytes)");
  if (batch == 0) return CS_OK;
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = stream ? static_cast<hipStream_t>(stream) : c->stream;
  int* piv = nullptr;
  HIPCHK(hipMalloc(&piv, sizeof(int) * (size_t)n * batch));
  launch_lu_solve(d_A, (size_t)lda * n, n, n + nrhs, lda, piv, n, nullptr, 0, 0, batch, d_info, st,
                  LU_KKT, batch);
  hipError_t e = hipGetLastError();
  hipError_t e2 = hipStreamSynchronize(st);
  hipFree(piv);
  if (e != hipSuccess || e2 != hipSuccess)
    return fail(CS_EDEVICE, std::string("cs_dense_solve_batched: ") +
                                hipGetErrorString(e != hipSuccess ? e : e2));
  return CS_OK;
}

extern "C" int cs_eigvals_batched(const cs_ctx* c, double* d_A, int32_t n, int32_t lda,
                                  int32_t batch, double* d_wr, double* d_wi, int32_t* d_info,
                                  void* stream) {
  if (!c || !d_A || !d_wr || !d_wi || n <= 0 || lda < n || batch < 0)
    return fail(CS_EINVAL, "cs_eigvals_batched: bad arguments");
  if (n > 1024) return fail(CS_EUNSUPPORTED, "cs_eigvals_batched: n > 1024");
  if (batch == 0) return CS_OK;
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = stream ? static_cast<hipStream_t>(stream) : c->stream;
  // the reduction's panel products: a temporary scratch of 64 n doubles per matrix
  double* scr = nullptr;
  const size_t scr_stride = eig_scratch_doubles(n);
  if (hipMalloc(&scr, sizeof(double) * scr_stride * (size_t)batch) != hipSuccess)
    return fail(CS_ENOMEM, "cs_eigvals_batched: scratch allocation failed");
  launch_eig(d_A, (size_t)lda * n, lda, nullptr, n, d_wr, d_wi, n, nullptr, batch, d_info, scr,
             scr_stride, st);
  const hipError_t e1 = hipGetLastError();
  const hipError_t e2 = hipStreamSynchronize(st);
  hipFree(scr);
  if (e1 != hipSuccess || e2 != hipSuccess)
    return fail(CS_EDEVICE, std::string("cs_eigvals_batched: ") +
                                hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  return CS_OK;
}

extern "C" int cs_kkt_at(cs_ctx* c, cs_net* n, const int32_t outage[2], int32_t iters,
                         double* K, double* x, double* lam, double* z, double* mu,
                         double* metrics, int32_t* status, int32_t* order) {
  if (!c || !n || !outage || iters < 0 || iters > 10000)
    return fail(CS_EINVAL, "cs_kkt_at: bad arguments");
  int rc = validate_host(n, outage, 1, nullptr);
  if (rc != CS_OK) return rc;
  HIPCHK(hipSetDevice(c->device));
  Plan p = plan_sizes(n, false);
  rc = bind_workspace(&c->ws, &c->ws_bytes, n, p, 1);
  if (rc != CS_OK) return rc;
  const Slots& s = p.s;
  const DevNet& D = n->d;
  hipStream_t st = c->stream;
  int* d_list = nullptr;
  HIPCHK(hipMalloc(&d_list, sizeof(int) * 2));
  hipMemcpy(d_list, outage, sizeof(int) * 2, hipMemcpyHostToDevice);
  const int big = iters + 100000;
  const double tol = 1e-8;
  launch_assign(s, 1, st);
  launch_islands(D, s, d_list, 1, st);
  launch_setup_k(D, s, 1, d_list, st);
  for (int it = 0; it < iters; ++it) {
    launch_opf_eval(D, s, 1, tol, big, st);
    launch_lu_solve(s.K, s.k_stride, s.nk, s.nk + 1, s.ldk, s.piv, std::max(s.nk, s.ny), s.st,
                    PH_IPM, 1, 1, nullptr, st);
    launch_opf_update(D, s, 1, 1e10, st);
  }
  launch_opf_eval(D, s, 1, tol, big, st);
  hipError_t e = hipStreamSynchronize(st);
  hipFree(d_list);
  if (e != hipSuccess) return fail(CS_EDEVICE, std::string("cs_kkt_at: ") + hipGetErrorString(e));
  SlotState S;
  HIPCHK(hipMemcpy(&S, s.st, sizeof(SlotState), hipMemcpyDeviceToHost));
  const int nk = s.nk;
  if (K) {
    std::vector<double> buf((size_t)nk * s.ldk);
    HIPCHK(hipMemcpy(buf.data(), s.K, sizeof(double) * buf.size(), hipMemcpyDeviceToHost));
    for (int r = 0; r < nk; ++r)
      for (int col = 0; col <= nk; ++col) K[(size_t)r * (nk + 1) + col] = buf[(size_t)r * s.ldk + col];
  }
  if (x) HIPCHK(hipMemcpy(x, s.x, sizeof(double) * s.nx, hipMemcpyDeviceToHost));
  if (lam) HIPCHK(hipMemcpy(lam, s.lam, sizeof(double) * s.neq, hipMemcpyDeviceToHost));
  if (z) HIPCHK(hipMemcpy(z, s.z, sizeof(double) * s.ni, hipMemcpyDeviceToHost));
  if (mu) HIPCHK(hipMemcpy(mu, s.mu, sizeof(double) * s.ni, hipMemcpyDeviceToHost));
  if (metrics) {
    for (int k = 0; k < 4; ++k) metrics[k] = S.metrics[k];
    metrics[4] = S.gamma;
    metrics[5] = S.singular;
    metrics[6] = S.f;
    metrics[7] = S.iters;
  }
  if (status) *status = (S.phase == PH_IPM) ? CS_OPF_MAXIT : S.status;
  if (order) *order = nk;
  return CS_OK;
}

extern "C" int cs_screen_detail(cs_ctx* c, cs_net* n, const int32_t* outages, int64_t N,
                                const cs_opts* opts, cs_result* out, double* vm, double* va,
                                double* pg, double* qg, double* eig_re, double* eig_im,
                                int32_t* n_eig) {
  if (!c || !n || N < 0 || (N > 0 && (!outages || !out || !vm || !va || !pg || !qg ||
                                      !eig_re || !eig_im || !n_eig)))
    return fail(CS_EINVAL, "cs_screen_detail: NULL argument or negative n");
  int rc = validate_host(n, outages, N, nullptr);
  if (rc != CS_OK) return rc;
  if (N == 0) return CS_OK;
  HIPCHK(hipSetDevice(c->device));
  const size_t nb = n->nb, ng = n->ng, na = (size_t)n->na;
  const size_t per = 2 * nb + 2 * ng + 2 * na;
  int* d_list = nullptr;
  cs_result* d_res = nullptr;
  double* d_det = nullptr;
  int* d_ne = nullptr;
  auto cleanup = [&]() {
    if (d_list) hipFree(d_list);
    if (d_res) hipFree(d_res);
    if (d_det) hipFree(d_det);
    if (d_ne) hipFree(d_ne);
  };
  if (hipMalloc(&d_list, sizeof(int) * 2 * N) != hipSuccess ||
      hipMalloc(&d_res, sizeof(cs_result) * N) != hipSuccess ||
      hipMalloc(&d_det, sizeof(double) * per * N) != hipSuccess ||
      hipMalloc(&d_ne, sizeof(int) * N) != hipSuccess) {
    cleanup();
    return fail(CS_ENOMEM, "cs_screen_detail: device allocation failed");
  }
  DetailOut det;
  det.vm = d_det;
  det.va = det.vm + nb * N;
  det.pg = det.va + nb * N;
  det.qg = det.pg + ng * N;
  det.eig_re = det.qg + ng * N;
  det.eig_im = det.eig_re + na * N;
  det.n_eig = d_ne;
  if (hipMemcpy(d_list, outages, sizeof(int) * 2 * N, hipMemcpyHostToDevice) != hipSuccess) {
    cleanup();
    return fail(CS_EDEVICE, "cs_screen_detail: copy to device failed");
  }
  rc = run_screen(c, n, d_list, N, nullptr, opts, d_res, nullptr, c->stream, nullptr, &det);
  if (rc == CS_OK) {
    const struct { double* h; const double* d; size_t cnt; } cp[] = {
        {vm, det.vm, nb * N}, {va, det.va, nb * N}, {pg, det.pg, ng * N},
        {qg, det.qg, ng * N}, {eig_re, det.eig_re, na * N}, {eig_im, det.eig_im, na * N}};
    bool ok = hipMemcpy(out, d_res, sizeof(cs_result) * N, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(n_eig, d_ne, sizeof(int) * N, hipMemcpyDeviceToHost) == hipSuccess;
    for (const auto& e : cp)
      ok = ok && hipMemcpy(e.h, e.d, sizeof(double) * e.cnt, hipMemcpyDeviceToHost) == hipSuccess;
    if (!ok) rc = fail(CS_EDEVICE, "cs_screen_detail: copy to host failed");
  }
  cleanup();
  return rc;
}

extern "C" int cs_dyn_at(cs_ctx* c, cs_net* n, const int32_t outage[2], const double* vm,
                         const double* va, const double* pg, const double* qg, double* A,
                         int32_t* n_states, double* eig_re, double* eig_im) {
  if (!c || !n || !outage || !vm || !va || !pg || !qg || !n_states)
    return fail(CS_EINVAL, "cs_dyn_at: NULL argument");
  int rc = validate_host(n, outage, 1, nullptr);
  if (rc != CS_OK) return rc;
  HIPCHK(hipSetDevice(c->device));
  Plan p = plan_sizes(n, false);
  rc = bind_workspace(&c->ws, &c->ws_bytes, n, p, 1);
  if (rc != CS_OK) return rc;
  const Slots& s = p.s;
  const DevNet& D = n->d;
  const int nb = n->nb, ng = n->ng;
  hipStream_t st = c->stream;
  int* d_list = nullptr;
  HIPCHK(hipMalloc(&d_list, sizeof(int) * 2));
  if (hipMemcpy(d_list, outage, sizeof(int) * 2, hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(d_list);
    return fail(CS_EDEVICE, "cs_dyn_at: copy to device failed");
  }
  launch_assign(s, 1, st);
  launch_islands(D, s, d_list, 1, st);
  launch_setup_k(D, s, 1, d_list, st);
  hipError_t e = hipStreamSynchronize(st);
  hipFree(d_list);
  if (e != hipSuccess) return fail(CS_EDEVICE, std::string("cs_dyn_at: ") + hipGetErrorString(e));
  SlotState S;
  HIPCHK(hipMemcpy(&S, s.st, sizeof(SlotState), hipMemcpyDeviceToHost));
  if (S.phase != PH_IPM)
    return fail(CS_EINVAL, "cs_dyn_at: the outage leaves no island with a generator to linearise");
  // the given operating point on the island's buses and in-service machines
  std::vector<double> x(s.nx);
  std::vector<uint8_t> bus_on(nb), gen_on(ng);
  HIPCHK(hipMemcpy(x.data(), s.x, sizeof(double) * s.nx, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(bus_on.data(), s.bus_on, nb, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(gen_on.data(), s.gen_on, ng, hipMemcpyDeviceToHost));
  for (int b = 0; b < nb; ++b)
    if (bus_on[b]) {
      if (!std::isfinite(va[b]) || !std::isfinite(vm[b]) || !(vm[b] > 0))
        return fail(CS_EINVAL, "cs_dyn_at: bus " + std::to_string(b) +
                                   " of the island needs a finite angle and a positive voltage");
      x[b] = va[b];
      x[nb + b] = vm[b];
    }
  for (int g = 0; g < ng; ++g)
    if (gen_on[g]) {
      if (!std::isfinite(pg[g]) || !std::isfinite(qg[g]))
        return fail(CS_EINVAL, "cs_dyn_at: generator " + std::to_string(g) + " needs finite P and Q");
      x[2 * nb + g] = pg[g];
      x[2 * nb + ng + g] = qg[g];
    }
  HIPCHK(hipMemcpy(s.x, x.data(), sizeof(double) * s.nx, hipMemcpyHostToDevice));
  S.phase = PH_DYNB;
  S.status = OPF_CONVERGED;
  S.job = 0;
  S.singular = 0;
  HIPCHK(hipMemcpy(s.st, &S, sizeof(SlotState), hipMemcpyHostToDevice));
  const int pstride = std::max(s.nk, s.ny);
  launch_dyn_assemble(D, s, 1, st);
  launch_lu_solve(s.K, s.k_stride, s.ny, s.nyc, s.ldy, s.piv, pstride, s.st, PH_DYNB, 1, 1,
                  nullptr, st, LU_DYN);
  launch_form_state(D, s, 1, st);
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipMemcpy(&S, s.st, sizeof(SlotState), hipMemcpyDeviceToHost));
  const int ns = S.n_states;
  *n_states = ns;
  if (A) {
    std::vector<double> a((size_t)s.lda_a * std::max(ns, 1));
    HIPCHK(hipMemcpy(a.data(), s.A, sizeof(double) * a.size(), hipMemcpyDeviceToHost));
    for (int r = 0; r < ns; ++r)
      for (int col = 0; col < ns; ++col) A[(size_t)r * ns + col] = a[(size_t)col * s.lda_a + r];
  }
  if (S.phase != PH_EIG)
    return fail(CS_EDEVICE, "cs_dyn_at: the algebraic system is singular or the state matrix is not finite");
  if (eig_re || eig_im) {
    launch_eig(s.A, s.a_stride, s.lda_a, nullptr, 0, s.wr, s.wi, s.na, s.st, 1, nullptr, s.K,
               s.k_stride, st);
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(&S, s.st, sizeof(SlotState), hipMemcpyDeviceToHost));
    if (S.qr_fail) return fail(CS_EDEVICE, "cs_dyn_at: QR iteration did not converge");
    if (eig_re) HIPCHK(hipMemcpy(eig_re, s.wr, sizeof(double) * ns, hipMemcpyDeviceToHost));
    if (eig_im) HIPCHK(hipMemcpy(eig_im, s.wi, sizeof(double) * ns, hipMemcpyDeviceToHost));
  }
  return CS_OK;
}

// ------------------------------------------------------------- risk variants
extern "C" void cs_risk_opts_default(cs_risk_opts* r) {
  if (!r) return;
  r->severity = CS_SEV_BINARY;
  r->zeta_ref = 0.05;
  r->n_cc = 0;
  r->cc_pairs = nullptr;
  r->cc_rate = nullptr;
}

// Device temporaries of one risk call, freed on every exit path.
struct RiskTemps {
  std::vector<void*> p;
  ~RiskTemps() {
    for (void* q : p) hipFree(q);
  }
  template <class T>
  T* take(size_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess) return nullptr;
    p.push_back(q);
    return static_cast<T*>(q);
  }
};

// Validate the list (and, when given, n_vals rate values) on the device,
// check the options on the host, and build the per-scenario severity
// weights and the common-cause table.
static int risk_prepare(const char* who, cs_ctx* c, cs_net* n, const int32_t* d_outages,
                        int64_t N, const cs_result* d_records, const double* d_vals,
                        long long n_vals, const cs_risk_opts* ro, hipStream_t st, RiskTemps& T,
                        double** w, double** cc) {
  const int n_comp = n->nl + n->ng + n->nd;
  cs_risk_opts r;
  cs_risk_opts_default(&r);
  if (ro) r = *ro;
  if (r.severity != CS_SEV_BINARY && r.severity != CS_SEV_DAMPING)
    return fail(CS_EINVAL, std::string(who) + ": severity must be CS_SEV_BINARY or CS_SEV_DAMPING");
  if (!(r.zeta_ref > 0) || !std::isfinite(r.zeta_ref))
    return fail(CS_EINVAL, std::string(who) + ": zeta_ref must be finite and > 0");
  if (r.n_cc < 0 || (r.n_cc > 0 && (!r.cc_pairs || !r.cc_rate)))
    return fail(CS_EINVAL, std::string(who) + ": common-cause pairs need cc_pairs and cc_rate");
  for (int64_t k = 0; k < r.n_cc; ++k) {
    const int a = r.cc_pairs[2 * k], b = r.cc_pairs[2 * k + 1];
    if (a < 0 || a >= n_comp || b < 0 || b >= n_comp || a == b)
      return fail(CS_EINVAL, std::string(who) + ": common-cause pair " + std::to_string(k) +
                                 " needs two distinct valid component ids");
    if (!(r.cc_rate[k] >= 0) || !std::isfinite(r.cc_rate[k]))
      return fail(CS_EINVAL, std::string(who) + ": common-cause rate " + std::to_string(k) +
                                 " must be finite and >= 0");
  }
  HIPCHK(hipMemsetAsync(c->d_counter, 0, sizeof(int), st));
  launch_validate(d_outages, N, n_comp, c->d_counter, st);
  if (d_vals) launch_validate_values(d_vals, n_vals, c->d_counter, st);
  HIPCHK(hipMemcpyAsync(c->h_counter, c->d_counter, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (*c->h_counter & 1) return fail(CS_EINVAL, std::string(who) + ": invalid outage row in the list");
  if (*c->h_counter & 2)
    return fail(CS_EINVAL, std::string(who) + ": every failure rate must be finite and >= 0");
  *w = T.take<double>(N);
  if (!*w) return fail(CS_ENOMEM, std::string(who) + ": device allocation failed");
  launch_sev_weights(d_records, N, r.severity, r.zeta_ref, *w, st);
  *cc = nullptr;
  if (r.n_cc > 0) {
    double* tab = T.take<double>((size_t)n_comp * n_comp);
    int* dp = T.take<int>(2 * (size_t)r.n_cc);
    double* dr = T.take<double>((size_t)r.n_cc);
    if (!tab || !dp || !dr) return fail(CS_ENOMEM, std::string(who) + ": device allocation failed");
    HIPCHK(hipMemsetAsync(tab, 0, sizeof(double) * (size_t)n_comp * n_comp, st));
    HIPCHK(hipMemcpyAsync(dp, r.cc_pairs, sizeof(int) * 2 * r.n_cc, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dr, r.cc_rate, sizeof(double) * r.n_cc, hipMemcpyHostToDevice, st));
    launch_cc_table(dp, dr, r.n_cc, n_comp, tab, st);
    *cc = tab;
  }
  return CS_OK;
}

extern "C" int cs_risk(cs_ctx* c, cs_net* n, const int32_t* d_outages, int64_t N,
                       const cs_result* d_records, const double* d_lambda,
                       const cs_risk_opts* ro, double* d_risk, void* stream) {
  if (!c || !n || N < 0 || !d_lambda || !d_risk || (N > 0 && (!d_outages || !d_records)))
    return fail(CS_EINVAL, "cs_risk: NULL argument or negative n");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = stream ? static_cast<hipStream_t>(stream) : c->stream;
  const int n_comp = n->nl + n->ng + n->nd;
  RiskTemps T;
  double *w = nullptr, *cc = nullptr;
  int rc = risk_prepare("cs_risk", c, n, d_outages, N, d_records, d_lambda, n_comp, ro, st, T,
                        &w, &cc);
  if (rc != CS_OK) return rc;
  launch_risk_weighted(d_outages, N, w, d_lambda, cc, n_comp, d_risk, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return CS_OK;
}

extern "C" int cs_risk_mc(cs_ctx* c, cs_net* n, const int32_t* d_outages, int64_t N,
                          const cs_result* d_records, const double* d_samples, int64_t M,
                          const cs_risk_opts* ro, double* d_risk, double* d_moments,
                          int32_t* d_rank_q, void* stream) {
  if (!c || !n || N < 0 || M <= 0 || !d_samples || (N > 0 && (!d_outages || !d_records)))
    return fail(CS_EINVAL, "cs_risk_mc: NULL argument, negative n or no samples");
  const int n_comp = n->nl + n->ng + n->nd;
  if (n_comp > 16384) return fail(CS_EUNSUPPORTED, "cs_risk_mc: more than 16384 components");
  if (M > (1ll << 24)) return fail(CS_EINVAL, "cs_risk_mc: more than 2^24 samples");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = stream ? static_cast<hipStream_t>(stream) : c->stream;
  RiskTemps T;
  double *w = nullptr, *cc = nullptr;
  int rc = risk_prepare("cs_risk_mc", c, n, d_outages, N, d_records, d_samples,
                        (long long)M * n_comp, ro, st, T, &w, &cc);
  if (rc != CS_OK) return rc;
  double* S1 = T.take<double>(n_comp);
  double* S2 = T.take<double>((size_t)n_comp * n_comp);
  double* C = T.take<double>(n_comp);
  double* R = d_risk ? d_risk : T.take<double>((size_t)M * n_comp);
  int* hist = d_rank_q ? T.take<int>((size_t)n_comp * n_comp) : nullptr;
  if (!S1 || !S2 || !C || !R || (d_rank_q && !hist))
    return fail(CS_ENOMEM, "cs_risk_mc: device allocation failed");
  HIPCHK(hipMemsetAsync(S2, 0, sizeof(double) * (size_t)n_comp * n_comp, st));
  launch_risk_split(d_outages, N, w, cc, n_comp, n_comp, S1, S2, C, st);
  launch_risk_mc_gemm(d_samples, M, n_comp, S1, S2, n_comp, C, R, st);
  if (hist) {
    HIPCHK(hipMemsetAsync(hist, 0, sizeof(int) * (size_t)n_comp * n_comp, st));
    launch_rank_hist(R, M, n_comp, hist, st);
  }
  if (d_moments || d_rank_q) launch_risk_summary(R, M, n_comp, hist, d_moments, d_rank_q, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return CS_OK;
}

// ---------------------------------------------------------------- N-3 lists
extern "C" int cs_screen3_device(cs_ctx* c, cs_net* n, const int32_t* d_outages, int64_t N,
                                 const double* d_lambda, const cs_opts* opts, cs_result* d_out,
                                 double* d_risk, void* stream) {
  return screen_device("cs_screen3_device", c, n, d_outages, N, d_lambda, opts, d_out, d_risk,
                       stream, false, 3);
}

extern "C" int cs_screen_n3_device(cs_ctx* c, cs_net* n, const int32_t* d_rows, int64_t N,
                                   const int32_t* d_sub, int64_t n_sub,
                                   const cs_result* d_sub_rec, const double* d_lambda,
                                   const cs_opts* opts, cs_result* d_out, double* d_risk,
                                   int64_t* n_solved, void* stream) {
  const char* who = "cs_screen_n3_device";
  if (!c || !n || N < 0 || n_sub < 0 || (N > 0 && (!d_rows || !d_out)) ||
      (n_sub > 0 && (!d_sub || !d_sub_rec)))
    return fail(CS_EINVAL, std::string(who) + ": NULL argument or negative size");
  if (d_risk && !d_lambda) return fail(CS_EINVAL, std::string(who) + ": risk requested without lambda");
  if (N > 0x7fffffffll) return fail(CS_EINVAL, std::string(who) + ": more than 2^31 - 1 rows");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = stream ? static_cast<hipStream_t>(stream) : c->stream;
  const int n_comp = n->nl + n->ng + n->nd;
  HIPCHK(hipMemsetAsync(c->d_counter, 0, sizeof(int), st));
  launch_validate(d_rows, N, n_comp, c->d_counter, st, 3);
  launch_validate(d_sub, n_sub, n_comp, c->d_counter, st, 2);
  if (d_lambda) launch_validate_rates(d_lambda, n_comp, c->d_counter, st);
  HIPCHK(hipMemcpyAsync(c->h_counter, c->d_counter, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (*c->h_counter & 1) return fail(CS_EINVAL, std::string(who) + ": invalid row in a list");
  if (*c->h_counter & 2)
    return fail(CS_EINVAL, std::string(who) + ": every failure rate must be finite and >= 0");
  if (n_solved) *n_solved = 0;
  if (N == 0) {
    if (d_risk) HIPCHK(hipMemsetAsync(d_risk, 0, sizeof(double) * n_comp, st));
    HIPCHK(hipStreamSynchronize(st));
    return CS_OK;
  }
  RiskTemps T;
  uint8_t* single = T.take<uint8_t>(n_comp);
  uint8_t* pair = T.take<uint8_t>((size_t)n_comp * n_comp);
  uint8_t* keep = T.take<uint8_t>(N);
  long long* idx = T.take<long long>(N);
  long long* cnt = T.take<long long>(1);
  const size_t sel_bytes = n3_select_bytes(N);
  void* sel = T.take<unsigned char>(sel_bytes);
  if (!single || !pair || !keep || !idx || !cnt || !sel || sel_bytes == 0)
    return fail(CS_ENOMEM, std::string(who) + ": device allocation failed");
  HIPCHK(hipMemsetAsync(single, 0, n_comp, st));
  HIPCHK(hipMemsetAsync(pair, 0, (size_t)n_comp * n_comp, st));
  launch_sub_severity(d_sub, n_sub, d_sub_rec, n_comp, single, pair, st);
  launch_n3_prune(d_rows, N, n_comp, single, pair, keep, st);
  if (n3_select(sel, sel_bytes, keep, N, idx, cnt, st) != 0)
    return fail(CS_EDEVICE, std::string(who) + ": compaction failed");
  long long k = 0;
  HIPCHK(hipMemcpyAsync(&k, cnt, sizeof(long long), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (n_solved) *n_solved = k;
  int* rows = T.take<int>(3 * (size_t)std::max<long long>(k, 1));
  cs_result* rec = T.take<cs_result>((size_t)std::max<long long>(k, 1));
  if (!rows || !rec) return fail(CS_ENOMEM, std::string(who) + ": device allocation failed");
  if (k > 0) {
    launch_gather_rows(d_rows, idx, k, rows, st);
    int rc = run_screen(c, n, rows, k, nullptr, opts, rec, nullptr, st, nullptr, nullptr, false, 3);
    if (rc != CS_OK) return rc;
  }
  launch_merge_n3(keep, N, rec, idx, k, d_out, st);
  if (d_risk)
    launch_risk(d_rows, N, reinterpret_cast<const uint8_t*>(d_out), (int)sizeof(cs_result),
                d_lambda, n_comp, d_risk, st, 3);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return CS_OK;
}
