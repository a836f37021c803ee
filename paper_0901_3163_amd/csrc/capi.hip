// extern "C" boundary of libdeflan (declared in include/deflan.h).
//
// Every entry point validates its arguments, converts between the caller's
// interleaved complex128 layout and the device's tiled site-major layout, runs
// the solver on the context's stream and maps C++ errors to DL_* status codes.
#include "engine.hpp"
#include "ptc.hpp"
#include "small.hpp"
#include "tsk.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <vector>

namespace dl {
const std::string& last_error();
}

using namespace dl;

namespace {

template <class F>
int guard(F&& f) {
  try {
    set_error("");
    return f();
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return DL_E_NOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return DL_E_INVALID;
  }
}

void need(bool ok, const char* msg) {
  if (!ok) fail(DL_E_INVALID, msg);
}

void use_device(dl_ctx* ctx) { DL_HIP(hipSetDevice(ctx->device)); }

// nfield fields in the caller's layout on lattice `lat` -> tiled device fields at t (pads zeroed).
void fields_in_lat(dl_op* op, const Lattice& lat, const double* p, int nfield, int mem, double2* t) {
  hipStream_t s = op->ctx->stream;
  zero(s, (long)nfield * lat.nc, t);
  const size_t bytes = (size_t)nfield * lat.V * kSpin * sizeof(double2);
  if (mem == DL_DEVICE) {
    pack_spinor(s, lat, reinterpret_cast<const double2*>(p), t, nfield);
  } else {
    DBuf<double2> stage((size_t)nfield * lat.V * kSpin);
    DL_HIP(hipMemcpyAsync(stage.get(), p, bytes, hipMemcpyHostToDevice, s));
    pack_spinor(s, lat, stage.get(), t, nfield);
    DL_HIP(hipStreamSynchronize(s));
  }
}

void fields_in_to(dl_op* op, const double* p, int nfield, int mem, double2* t) {
  fields_in_lat(op, op->lat, p, nfield, mem, t);
}

DBuf<double2> fields_in(dl_op* op, const double* p, int nfield, int mem) {
  DBuf<double2> t((size_t)nfield * op->lat.nc);
  fields_in_to(op, p, nfield, mem, t.get());
  return t;
}

void fields_out_lat(dl_op* op, const Lattice& lat, const double2* t, double* p, int nfield, int mem) {
  hipStream_t s = op->ctx->stream;
  const size_t bytes = (size_t)nfield * lat.V * kSpin * sizeof(double2);
  if (mem == DL_DEVICE) {
    unpack_spinor(s, lat, t, reinterpret_cast<double2*>(p), nfield);
  } else {
    DBuf<double2> stage((size_t)nfield * lat.V * kSpin);
    unpack_spinor(s, lat, t, stage.get(), nfield);
    DL_HIP(hipMemcpyAsync(p, stage.get(), bytes, hipMemcpyDeviceToHost, s));
  }
  DL_HIP(hipStreamSynchronize(s));
}

void fields_out(dl_op* op, const double2* t, double* p, int nfield, int mem) {
  fields_out_lat(op, op->lat, t, p, nfield, mem);
}

uint64_t fnv(uint64_t h, const void* data, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

dl_first_opts first_defaults(const dl_first_opts* o) {
  dl_first_opts d{};
  d.eig_tol = 1e-12;
  d.past_conv_factor = 2.0;
  d.max_mvp = 1000000;
  d.reorth = DL_REORTH_FULL;
  d.reorth_period = 1;
  if (o) {
    if (o->eig_tol > 0) d.eig_tol = o->eig_tol;
    if (o->past_conv_factor > 0) d.past_conv_factor = o->past_conv_factor;
    if (o->max_mvp > 0) d.max_mvp = o->max_mvp;
    need(o->reorth == DL_REORTH_FULL || o->reorth == DL_REORTH_KEPT, "reorth must be DL_REORTH_FULL or DL_REORTH_KEPT");
    need(o->reorth_period >= 0, "reorth_period must be >= 0");
    d.reorth = o->reorth;
    if (o->reorth_period > 0) d.reorth_period = o->reorth_period;
  }
  return d;
}

// inner_drop and reliable_every stay 0 when the caller leaves them at 0: the batched solver
// resolves them by storage and solver (and knows which ones the caller set)
dl_next_opts next_defaults(const dl_next_opts* o) {
  dl_next_opts d{};
  d.storage = DL_FP64;
  d.reliable_every = 0;  // resolved below by storage and solver
  d.batched = 0;
  d.x0_given = 0;
  d.max_mvp = 1000000;
  d.inner_drop = 0.0;  // resolved below by storage
  if (o) {
    d.storage = o->storage;
    if (o->reliable_every != 0) d.reliable_every = o->reliable_every;  // < 0: no reliable updates
    d.batched = o->batched;
    d.x0_given = o->x0_given;
    if (o->max_mvp > 0) d.max_mvp = o->max_mvp;
    d.net = o->net;
    d.graph = o->graph;
    if (o->inner_drop != 0.0) d.inner_drop = o->inner_drop;
    d.eig_storage = o->eig_storage;
    d.net_prec = o->net_prec;
    d.method = o->method;
    d.minres_window = o->minres_window;
  }
  if (d.net_prec == 0) d.net_prec = DL_FP32;
  return d;
}

// host complex128 weights <-> device FP32 complex weights
void weights_to_device(dl_net* net, const double* w) {
  const int nw = net_num_weights();
  std::vector<float2> h(nw);
  for (int i = 0; i < nw; ++i) {
    if (!std::isfinite(w[2 * i]) || !std::isfinite(w[2 * i + 1])) fail(DL_E_NONFINITE, "non-finite weight");
    h[i] = make_float2((float)w[2 * i], (float)w[2 * i + 1]);
  }
  DL_HIP(hipMemcpyAsync(net->W.get(), h.data(), nw * sizeof(float2), hipMemcpyHostToDevice, net->ctx->stream));
  DL_HIP(hipStreamSynchronize(net->ctx->stream));
}

void weights_to_host(const float2* d, double* w, hipStream_t s) {
  const int nw = net_num_weights();
  std::vector<float2> h(nw);
  DL_HIP(hipMemcpyAsync(h.data(), d, nw * sizeof(float2), hipMemcpyDeviceToHost, s));
  DL_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < nw; ++i) {
    w[2 * i] = h[i].x;
    w[2 * i + 1] = h[i].y;
  }
}

// The caller's residual-history requests (input fields of dl_stats), taken before a solve
// overwrites the entries, and given back with the points afterwards.
struct HistoryReq {
  std::vector<double*> ptr;
  History h;
  HistoryReq(const dl_stats* st, int n) : ptr(n, nullptr), h(n) {
    if (!st) return;
    for (int r = 0; r < n; ++r)
      if (st[r].history && st[r].history_cap > 0) {
        ptr[r] = st[r].history;
        h.cap[r] = st[r].history_cap;
      }
  }
  History* get() { return h.any() ? &h : nullptr; }
  void write(dl_stats* st, int n) const {
    if (!st) return;
    for (int r = 0; r < n; ++r) {
      st[r].history = ptr[r];
      st[r].history_cap = ptr[r] ? h.cap[r] : 0;
      st[r].history_len = ptr[r] ? (int)(h.pts[r].size() / 2) : 0;
      if (ptr[r] && !h.pts[r].empty()) std::memcpy(ptr[r], h.pts[r].data(), h.pts[r].size() * sizeof(double));
    }
  }
};

void check_net_op(const dl_net* net, const dl_op* op) {
  need(net->ctx == op->ctx, "network and operator belong to different contexts");
  need(!op->lat.eo, "the network works on whole-lattice fields (not on an even-odd operator)");
}

}  // namespace

extern "C" {

const char* dl_last_error(void) { return dl::last_error().c_str(); }

int dl_version(void) { return 200; }

int dl_ctx_create(int device, void* hip_stream, dl_ctx** out) {
  return guard([&] {
    need(out != nullptr, "out is NULL");
    int ndev = 0;
    DL_HIP(hipGetDeviceCount(&ndev));
    need(device >= 0 && device < ndev, "device index out of range");
    auto* c = new dl_ctx();
    try {
      c->device = device;
      DL_HIP(hipSetDevice(device));
      if (hip_stream) {
        c->stream = static_cast<hipStream_t>(hip_stream);
      } else {
        DL_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
      }
      void* pin = nullptr;
      DL_HIP(hipHostMalloc(&pin, 4096 * sizeof(double), hipHostMallocDefault));
      c->pinned = static_cast<double*>(pin);
      noalloc_init(device);  // device address of the no-allocation scratch array
    } catch (...) {
      if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
      delete c;
      throw;
    }
    *out = c;
    return DL_OK;
  });
}

void dl_ctx_destroy(dl_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->timers.collect();
  eo_release(ctx->stream);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  dl::dmem_trim(ctx->device);
  delete ctx;
}

int dl_ctx_sync(dl_ctx* ctx) {
  return guard([&] {
    need(ctx != nullptr, "ctx is NULL");
    use_device(ctx);
    DL_HIP(hipStreamSynchronize(ctx->stream));
    return DL_OK;
  });
}

int dl_timing(dl_ctx* ctx, int enable) {
  return guard([&] {
    need(ctx != nullptr, "ctx is NULL");
    use_device(ctx);
    ctx->timers.reset();
    ctx->timers.enabled = enable != 0;
    return DL_OK;
  });
}

int dl_kernel_time(dl_ctx* ctx, const char* name, long* launches, double* total_ms, double* bytes) {
  return guard([&] {
    need(ctx && name && launches && total_ms, "NULL argument");
    use_device(ctx);
    int id = -1;
    if (!std::strcmp(name, "wilson")) id = T_WILSON;
    else if (!std::strcmp(name, "tsk_dots")) id = T_TSK_DOTS;
    else if (!std::strcmp(name, "tsk_update")) id = T_TSK_UPDATE;
    else if (!std::strcmp(name, "small")) id = T_SMALL;
    else if (!std::strcmp(name, "wilson64")) id = T_WILSON64;
    need(id >= 0, "unknown kernel family");
    ctx->timers.collect();
    *launches = ctx->timers.launches[id];
    *total_ms = ctx->timers.ms[id];
    if (bytes) *bytes = ctx->timers.bytes[id];
    return DL_OK;
  });
}

int dl_op_create(dl_ctx* ctx, const int dims[4], const double* links, int mem, double kappa, int kind, dl_op** out) {
  return guard([&] {
    need(ctx && dims && links && out, "NULL argument");
    need(mem == DL_HOST || mem == DL_DEVICE, "mem must be DL_HOST or DL_DEVICE");
    const int base = kind & ~DL_EVEN_ODD;
    const bool eo = (kind & DL_EVEN_ODD) != 0;
    need(base == DL_MDAGM || base == DL_G5M, "kind must be DL_MDAGM or DL_G5M, optionally with DL_EVEN_ODD");
    need(std::isfinite(kappa), "kappa must be finite");
    use_device(ctx);
    auto* op = new dl_op();
    try {
      op->ctx = ctx;
      op->lat = eo ? make_lattice_eo(dims) : make_lattice(dims);
      op->kappa = kappa;
      op->kind = base;
      const Lattice lat = make_lattice(dims);  // the links cover the whole lattice
      hipStream_t s = ctx->stream;
      op->U.alloc(lat.nl);
      zero(s, lat.nl, op->U.get());
      const size_t bytes = (size_t)lat.V * kLinkC * sizeof(double2);
      if (mem == DL_DEVICE) {
        pack_links(s, lat, reinterpret_cast<const double2*>(links), op->U.get());
      } else {
        DBuf<double2> stage((size_t)lat.V * kLinkC);
        DL_HIP(hipMemcpyAsync(stage.get(), links, bytes, hipMemcpyHostToDevice, s));
        pack_links(s, lat, stage.get(), op->U.get());
        DL_HIP(hipStreamSynchronize(s));
      }
      // every link as stored on the device, whatever memory it came from
      const uint64_t lh = field_hash(s, lat.nl, op->U.get());
      uint64_t h = 1469598103934665603ull;
      h = fnv(h, dims, 4 * sizeof(int));
      h = fnv(h, &kappa, sizeof(double));
      h = fnv(h, &kind, sizeof(int));
      h = fnv(h, &lh, sizeof(lh));
      op->fingerprint = h;
    } catch (...) {
      delete op;
      throw;
    }
    *out = op;
    return DL_OK;
  });
}

void dl_op_destroy(dl_op* op) {
  if (!op) return;
  (void)hipSetDevice(op->ctx->device);
  (void)hipStreamSynchronize(op->ctx->stream);
  delete op;
}

long dl_op_size(const dl_op* op) { return op ? 12 * op->lat.V : 0; }

int dl_eo_prepare(dl_op* op, const double* b, double* bhat, int mem) {
  return guard([&] {
    need(op && b && bhat, "NULL argument");
    need(op->lat.eo, "dl_eo_prepare needs an operator created with DL_EVEN_ODD");
    need(mem == DL_HOST || mem == DL_DEVICE, "mem must be DL_HOST or DL_DEVICE");
    use_device(op->ctx);
    hipStream_t s = op->ctx->stream;
    const Lattice full = make_lattice(op->lat.L);
    DBuf<double2> bt(full.nc), be(op->lat.nc), bo(op->lat.nc), bh(op->lat.nc);
    fields_in_lat(op, full, b, 1, mem, bt.get());
    eo_split(s, full, bt.get(), be.get(), 0, 1);
    eo_split(s, full, bt.get(), bo.get(), 1, 1);
    eo_hop_f64(s, op->lat, op->U.get(), op->kappa, 0, bo.get(), be.get(), bh.get());  // b_e + kappa D_eo b_o
    fields_out(op, bh.get(), bhat, 1, mem);
    return DL_OK;
  });
}

int dl_eo_reconstruct(dl_op* op, const double* b, const double* xe, double* x, int mem) {
  return guard([&] {
    need(op && b && xe && x, "NULL argument");
    need(op->lat.eo, "dl_eo_reconstruct needs an operator created with DL_EVEN_ODD");
    need(mem == DL_HOST || mem == DL_DEVICE, "mem must be DL_HOST or DL_DEVICE");
    use_device(op->ctx);
    hipStream_t s = op->ctx->stream;
    const Lattice full = make_lattice(op->lat.L);
    DBuf<double2> bt(full.nc), bo(op->lat.nc), xo(op->lat.nc), xt(full.nc);
    DBuf<double2> xet = fields_in(op, xe, 1, mem);
    fields_in_lat(op, full, b, 1, mem, bt.get());
    eo_split(s, full, bt.get(), bo.get(), 1, 1);
    eo_hop_f64(s, op->lat, op->U.get(), op->kappa, 1, xet.get(), bo.get(), xo.get());  // b_o + kappa D_oe x_e
    zero(s, full.nc, xt.get());
    eo_merge(s, full, xet.get(), xt.get(), 0, 1);
    eo_merge(s, full, xo.get(), xt.get(), 1, 1);
    fields_out_lat(op, full, xt.get(), x, 1, mem);
    return DL_OK;
  });
}

int dl_op_fingerprint(const dl_op* op, unsigned long long* out) {
  return guard([&] {
    need(op && out, "NULL argument");
    *out = (unsigned long long)op->fingerprint;
    return DL_OK;
  });
}

int dl_apply(dl_op* op, int which, const double* in, double* out, int mem) {
  return guard([&] {
    need(op && in && out, "NULL argument");
    need(which >= 0 && which <= 3, "which must be one of DL_APPLY_*");
    need(mem == DL_HOST || mem == DL_DEVICE, "mem must be DL_HOST or DL_DEVICE");
    need(in != out, "in and out may not alias");
    use_device(op->ctx);
    DBuf<double2> t = fields_in(op, in, 1, mem);
    DBuf<double2> r(op->lat.nc), tmp(op->lat.nc);
    zero(op->ctx->stream, op->lat.nc, r.get());
    zero(op->ctx->stream, op->lat.nc, tmp.get());
    if (which == DL_APPLY_MDAGM) {
      apply_wilson(op, 0, t.get(), tmp.get());
      apply_wilson(op, 1, tmp.get(), r.get());
    } else {
      apply_wilson(op, which, t.get(), r.get());
    }
    fields_out(op, r.get(), out, 1, mem);
    return DL_OK;
  });
}

int dl_solve_first(dl_op* op, const double* b, double* x, int mem, int m, int k, double tol,
                   const dl_first_opts* opts, dl_eig** eig_out, dl_stats* stats) {
  return guard([&] {
    need(op && b && x, "NULL argument");
    need(mem == DL_HOST || mem == DL_DEVICE, "mem must be DL_HOST or DL_DEVICE");
    need(k >= 0 && m > k, "need 0 <= k < m");
    need((long)m <= 12 * op->lat.V, "m exceeds the vector length");
    need(m <= 510, "m must be <= 510");
    need(tol > 0 && std::isfinite(tol), "tol must be positive");
    use_device(op->ctx);
    const dl_first_opts o = first_defaults(opts);
    DBuf<double2> bt = fields_in(op, b, 1, mem);
    DBuf<double2> xt(op->lat.nc);
    zero(op->ctx->stream, op->lat.nc, xt.get());
    dl_eig* e = nullptr;
    HistoryReq hr(stats, 1);
    const int rc = solve_first(op, bt.get(), xt.get(), m, k, tol, o, eig_out ? &e : nullptr, stats, hr.get());
    fields_out(op, xt.get(), x, 1, mem);
    hr.write(stats, 1);
    if (eig_out) *eig_out = e;
    return rc;
  });
}

int dl_solve_next(dl_op* op, const dl_eig* eig, int nrhs, const double* B, double* X, int mem, double tol,
                  const dl_next_opts* opts, dl_stats* stats) {
  return guard([&] {
    need(op != nullptr, "op is NULL");
    need(nrhs >= 0, "nrhs must be >= 0");
    if (nrhs == 0) return DL_OK;
    need(B && X, "NULL argument");
    need(mem == DL_HOST || mem == DL_DEVICE, "mem must be DL_HOST or DL_DEVICE");
    need(tol > 0 && std::isfinite(tol), "tol must be positive");
    const dl_next_opts o = next_defaults(opts);
    need(o.storage == DL_FP64 || o.storage == DL_FP32 || o.storage == DL_BF16,
         "storage must be DL_FP64, DL_FP32 or DL_BF16");
    need(!(o.storage != DL_FP64 && !o.batched), "DL_FP32 and DL_BF16 storage run through the batched path (batched = 1)");
    need(!(o.batched && o.storage == DL_FP64), "the batched path stores Krylov vectors in DL_FP32 or DL_BF16");
    need(o.inner_drop == 0.0 || (o.inner_drop > 0.0 && o.inner_drop < 1.0), "inner_drop must be in (0, 1)");
    need(!o.net || o.batched, "the learned initial guess runs on the batched path (batched = 1)");
    need(o.eig_storage == DL_FP64 || o.eig_storage == DL_FP32 || o.eig_storage == DL_BF16,
         "eig_storage must be DL_FP64, DL_FP32 or DL_BF16");
    need(o.eig_storage == DL_FP64 || o.batched, "lowered eigenvectors are read by the batched path (batched = 1)");
    need(o.net_prec == DL_FP32 || o.net_prec == DL_BF16, "net_prec must be DL_FP32 or DL_BF16");
    need(o.method == DL_METHOD_DEFAULT || o.method == DL_METHOD_CG, "method must be DL_METHOD_DEFAULT or DL_METHOD_CG");
    need(o.method == DL_METHOD_DEFAULT || !o.batched, "method DL_METHOD_CG runs on the FP64 one-rhs path (batched = 0)");
    need(!(o.net && o.x0_given), "x0_given and a learned initial guess exclude each other");
    need(o.minres_window <= 64, "minres_window must be at most 64");
    if (o.net) check_net_op(o.net, op);
    use_device(op->ctx);
    if (eig && (eig->fingerprint != op->fingerprint || eig->kind != op->kind))
      fail(DL_E_MISMATCH, "eigenvector handle was built for a different operator");
    DBuf<double2> bt = fields_in(op, B, nrhs, mem);
    DBuf<double2> xt = o.x0_given ? fields_in(op, X, nrhs, mem) : DBuf<double2>((size_t)nrhs * op->lat.nc);
    if (!o.x0_given) zero(op->ctx->stream, (long)nrhs * op->lat.nc, xt.get());
    HistoryReq hr(stats, nrhs);
    const int rc = o.batched ? solve_next_batched(op, eig, nrhs, bt.get(), xt.get(), tol, o, stats, hr.get())
                             : solve_next(op, eig, nrhs, bt.get(), xt.get(), tol, o, stats, hr.get());
    fields_out(op, xt.get(), X, nrhs, mem);
    hr.write(stats, nrhs);
    return rc;
  });
}

int dl_apply_batched(dl_op* op, int which, int prec, int nrhs, const double* in, double* out, int mem) {
  return guard([&] {
    need(op != nullptr, "op is NULL");
    need(which >= 0 && which <= 2, "which must be DL_APPLY_M, DL_APPLY_MDAG or DL_APPLY_G5M");
    need(prec == DL_FP64 || prec == DL_FP32 || prec == DL_BF16, "prec must be DL_FP64, DL_FP32 or DL_BF16");
    need(nrhs >= 0, "nrhs must be >= 0");
    if (nrhs == 0) return DL_OK;
    need(in && out, "NULL argument");
    need(in != out, "in and out may not alias");
    need(mem == DL_HOST || mem == DL_DEVICE, "mem must be DL_HOST or DL_DEVICE");
    use_device(op->ctx);
    hipStream_t s = op->ctx->stream;
    const Lattice& lat = op->lat;
    const long n = (long)nrhs * lat.nc;
    DBuf<double2> t = fields_in(op, in, nrhs, mem);
    DBuf<double2> r(n);
    const WilsonCfg cfg = wilson_cfg(op, prec, nrhs);
    if (prec == DL_FP64) {
      wilson_batched<double>(s, lat, op->U.get(), op->kappa, which, t.get(), r.get(), lat.nc, nrhs, 0, nullptr,
                             nullptr, nullptr, cfg);
    } else if (prec == DL_FP32) {
      DBuf<float2> a32(n), b32(n);
      round_f32(s, n, t.get(), a32.get());
      wilson_batched<float>(s, lat, op_links32_public(op), op->kappa, which, a32.get(), b32.get(), lat.nc, nrhs, 0,
                            nullptr, nullptr, nullptr, cfg);
      widen_f64(s, n, b32.get(), r.get());
      DL_HIP(hipStreamSynchronize(s));
    } else {
      DBuf<bf2> a16(n), b16(n);
      round_bf16(s, n, t.get(), a16.get());
      wilson_batched<float>(s, lat, op_links32_public(op), op->kappa, which, a16.get(), b16.get(), lat.nc, nrhs, 0,
                            nullptr, nullptr, nullptr, cfg);
      widen_bf16(s, n, b16.get(), r.get());
      DL_HIP(hipStreamSynchronize(s));
    }
    fields_out(op, r.get(), out, nrhs, mem);
    return DL_OK;
  });
}

int dl_solve_next_multi(dl_ctx* ctx, int nitems, const dl_batch_item* items, int mem, const dl_next_opts* opts,
                        dl_stats* stats) {
  return guard([&] {
    need(ctx != nullptr, "ctx is NULL");
    need(nitems >= 0, "nitems must be >= 0");
    if (nitems == 0) return DL_OK;
    need(items != nullptr, "items is NULL");
    need(mem == DL_HOST || mem == DL_DEVICE, "mem must be DL_HOST or DL_DEVICE");
    need(items[0].op != nullptr, "item op is NULL");
    dl_next_opts o = next_defaults(opts);
    if (!opts) {
      o.storage = DL_FP32;
      o.batched = 1;
    }
    need((o.storage == DL_FP32 || o.storage == DL_BF16) && o.batched,
         "the multi-lattice batch runs the batched path (DL_FP32 or DL_BF16, batched = 1)");
    need(o.inner_drop == 0.0 || (o.inner_drop > 0.0 && o.inner_drop < 1.0), "inner_drop must be in (0, 1)");
    need(!o.net, "the learned initial guess takes one operator per batch (dl_solve_next)");
    need(o.minres_window <= 64, "minres_window must be at most 64");
    need(o.eig_storage == DL_FP64 || o.eig_storage == DL_FP32 || o.eig_storage == DL_BF16,
         "eig_storage must be DL_FP64, DL_FP32 or DL_BF16");
    use_device(ctx);
    std::vector<MultiItem> mi;
    std::vector<int> src;  // item index of each batch entry
    long total = 0;
    int kind = -1;
    for (int i = 0; i < nitems; ++i) {
      const dl_batch_item& it = items[i];
      need(it.op != nullptr, "item op is NULL");
      need(it.op->ctx == ctx, "every operator of the batch must belong to ctx");
      need(!it.op->lat.eo, "the multi-lattice batch takes whole-lattice operators (no DL_EVEN_ODD)");
      need(it.nrhs >= 0, "item nrhs must be >= 0");
      need(it.tol > 0 && std::isfinite(it.tol), "item tol must be positive");
      if (kind < 0) kind = it.op->kind;
      need(it.op->kind == kind, "every operator of the batch must have the same kind");
      if (it.eig && (it.eig->fingerprint != it.op->fingerprint || it.eig->kind != it.op->kind))
        fail(DL_E_MISMATCH, "eigenvector handle was built for a different operator");
      if (it.nrhs == 0) continue;
      need(it.B && it.X, "item B or X is NULL");
      mi.push_back(MultiItem{it.op, it.eig, it.nrhs, it.tol});
      src.push_back(i);
      total += (long)it.nrhs * it.op->lat.nc;
    }
    if (mi.empty()) return DL_OK;
    DBuf<double2> bt((size_t)total), xt((size_t)total);
    long off = 0;
    for (size_t j = 0; j < mi.size(); ++j) {
      const dl_batch_item& it = items[src[j]];
      fields_in_to(it.op, it.B, it.nrhs, mem, bt.get() + off);
      if (o.x0_given) fields_in_to(it.op, it.X, it.nrhs, mem, xt.get() + off);
      off += (long)it.nrhs * it.op->lat.nc;
    }
    std::vector<dl_stats> st;
    long nst = 0;
    for (const auto& m : mi) nst += m.nrhs;
    st.resize(nst);
    HistoryReq hr(stats, (int)nst);
    const int rc = solve_next_multi(mi, bt.get(), xt.get(), o, st.data(), hr.get());
    off = 0;
    long r = 0;
    for (size_t j = 0; j < mi.size(); ++j) {
      const dl_batch_item& it = items[src[j]];
      fields_out(it.op, xt.get() + off, it.X, it.nrhs, mem);
      off += (long)it.nrhs * it.op->lat.nc;
    }
    if (stats) {
      // stats in item order, nrhs entries per item (items with nrhs = 0 have none)
      for (size_t j = 0; j < mi.size(); ++j)
        for (int q = 0; q < mi[j].nrhs; ++q, ++r) stats[r] = st[r];
      hr.write(stats, (int)nst);
    }
    return rc;
  });
}

int dl_bench_wilson(dl_op* op, int which, int prec, int nrhs, int reps, double* avg_ms, double* bytes) {
  return guard([&] {
    need(op && avg_ms, "NULL argument");
    need(which >= 0 && which <= 2, "which must be DL_APPLY_M, DL_APPLY_MDAG or DL_APPLY_G5M");
    need(prec == DL_FP64 || prec == DL_FP32 || prec == DL_BF16, "prec must be DL_FP64, DL_FP32 or DL_BF16");
    need(nrhs >= 1 && nrhs <= 256 && reps >= 1, "need 1 <= nrhs <= 256 and reps >= 1");
    use_device(op->ctx);
    hipStream_t s = op->ctx->stream;
    const Lattice& lat = op->lat;
    const long n = (long)nrhs * lat.nc;
    const WilsonCfg cfg = wilson_cfg(op, prec, nrhs);
    hipEvent_t a, b;
    DL_HIP(hipEventCreate(&a));
    DL_HIP(hipEventCreate(&b));
    double bb;
    float ms = 0.f;
    if (prec == DL_FP64) {
      DBuf<double2> in(n), out(n);
      zero(s, n, in.get());
      wilson_batched<double>(s, lat, op->U.get(), op->kappa, which, in.get(), out.get(), lat.nc, nrhs, 0, nullptr,
                             nullptr, nullptr, cfg);
      DL_HIP(hipEventRecord(a, s));
      for (int i = 0; i < reps; ++i)
        wilson_batched<double>(s, lat, op->U.get(), op->kappa, which, in.get(), out.get(), lat.nc, nrhs, 0,
                               nullptr, nullptr, nullptr, cfg);
      DL_HIP(hipEventRecord(b, s));
      DL_HIP(hipEventSynchronize(b));
      bb = (double)lat.V * (576.0 + 384.0 * nrhs);
    } else if (prec == DL_BF16) {
      DBuf<bf2> in(n), out(n);
      zero(s, n / 4, reinterpret_cast<double2*>(in.get()));  // n bf2 = n/4 double2 (nc is a multiple of 4)
      const float2* U32 = op_links32_public(op);
      wilson_batched<float>(s, lat, U32, op->kappa, which, in.get(), out.get(), lat.nc, nrhs, 0, nullptr, nullptr,
                            nullptr, cfg);
      DL_HIP(hipEventRecord(a, s));
      for (int i = 0; i < reps; ++i)
        wilson_batched<float>(s, lat, U32, op->kappa, which, in.get(), out.get(), lat.nc, nrhs, 0, nullptr,
                              nullptr, nullptr, cfg);
      DL_HIP(hipEventRecord(b, s));
      DL_HIP(hipEventSynchronize(b));
      bb = (double)lat.V * (288.0 + 96.0 * nrhs);
    } else {
      DBuf<float2> in(n), out(n);
      zero(s, n / 2, reinterpret_cast<double2*>(in.get()));  // n float2 = n/2 double2 (nc is even)
      const float2* U32 = op_links32_public(op);
      wilson_batched<float>(s, lat, U32, op->kappa, which, in.get(), out.get(), lat.nc, nrhs, 0, nullptr, nullptr,
                            nullptr, cfg);
      DL_HIP(hipEventRecord(a, s));
      for (int i = 0; i < reps; ++i)
        wilson_batched<float>(s, lat, U32, op->kappa, which, in.get(), out.get(), lat.nc, nrhs, 0, nullptr,
                              nullptr, nullptr, cfg);
      DL_HIP(hipEventRecord(b, s));
      DL_HIP(hipEventSynchronize(b));
      bb = (double)lat.V * (288.0 + 192.0 * nrhs);
    }
    DL_HIP(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (lat.eo) {
      // Mhat: both half stages read every link once; per rhs the input half field twice, the odd
      // intermediate (arithmetic precision) written and read once, the output written once
      const double linkb = prec == DL_FP64 ? 576.0 : 288.0, tmpb = prec == DL_FP64 ? 192.0 : 96.0;
      const double spb = prec == DL_FP64 ? 192.0 : prec == DL_FP32 ? 96.0 : 48.0;
      bb = 2.0 * (2.0 * lat.V) * linkb + (double)nrhs * lat.V * (3.0 * spb + 2.0 * tmpb);
    }
    *avg_ms = ms / reps;
    if (bytes) *bytes = bb;
    return DL_OK;
  });
}

int dl_bench_copy(dl_ctx* ctx, long bytes, int reps, double* avg_ms) {
  return guard([&] {
    need(ctx && avg_ms, "NULL argument");
    need(bytes >= 16 && reps >= 1, "need bytes >= 16 and reps >= 1");
    use_device(ctx);
    hipStream_t s = ctx->stream;
    const long n = bytes / 16;
    DBuf<double2> a(n), b(n);
    zero(s, n, a.get());
    copy(s, n, a.get(), b.get());
    hipEvent_t e0, e1;
    DL_HIP(hipEventCreate(&e0));
    DL_HIP(hipEventCreate(&e1));
    DL_HIP(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i) copy(s, n, a.get(), b.get());
    DL_HIP(hipEventRecord(e1, s));
    DL_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    DL_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = ms / reps;
    return DL_OK;
  });
}

int dl_tune_wilson(dl_op* op, int prec, int nrhs, int reps, int* variant, int* order, double* best_us) {
  return guard([&] {
    need(op != nullptr, "op is NULL");
    need(prec == DL_FP64 || prec == DL_FP32 || prec == DL_BF16, "prec must be DL_FP64, DL_FP32 or DL_BF16");
    need(nrhs >= 1 && nrhs <= 256 && reps >= 1, "need 1 <= nrhs <= 256 and reps >= 1");
    use_device(op->ctx);
    double us = 0.0;
    const WilsonCfg c = tune_wilson(op, prec, nrhs, reps, &us);
    if (variant) *variant = c.variant;
    if (order) *order = c.order;
    if (best_us) *best_us = us;
    return DL_OK;
  });
}

int dl_tune_tsk(dl_ctx* ctx, int kind, long n, int nv, int nw, int reps, int* grid, int* tile, double* best_us) {
  return guard([&] {
    need(ctx != nullptr, "ctx is NULL");
    need(kind >= 0 && kind < TK_COUNT, "unknown contraction kind");
    need(n >= 1 && nv >= 1 && nw >= 1 && reps >= 1, "need n, nv, nw, reps >= 1");
    use_device(ctx);
    double us = 0.0;
    const TskCfg c = tsk_tune(ctx->stream, kind, n, nv, nw, reps, &us);
    if (grid) *grid = c.grid;
    if (tile) *tile = c.tile;
    if (best_us) *best_us = us;
    return DL_OK;
  });
}

int dl_net_num_weights(void) { return net_num_weights(); }

int dl_net_create(dl_ctx* ctx, const double* weights, dl_net** out) {
  return guard([&] {
    need(ctx && weights && out, "NULL argument");
    use_device(ctx);
    auto* net = new dl_net();
    try {
      net->ctx = ctx;
      const int nw = net_num_weights();
      net->W.alloc(nw);
      net->G.alloc(nw);
      net->Wt.alloc(nw);
      net->m.alloc(2 * nw);
      net->v.alloc(2 * nw);
      net_reset_adam(net);
      weights_to_device(net, weights);
    } catch (...) {
      delete net;
      throw;
    }
    *out = net;
    return DL_OK;
  });
}

int dl_net_get_weights(const dl_net* net, double* weights) {
  return guard([&] {
    need(net && weights, "NULL argument");
    use_device(net->ctx);
    weights_to_host(net->W.get(), weights, net->ctx->stream);
    return DL_OK;
  });
}

int dl_net_set_weights(dl_net* net, const double* weights) {
  return guard([&] {
    need(net && weights, "NULL argument");
    use_device(net->ctx);
    weights_to_device(net, weights);
    net_reset_adam(net);
    DL_HIP(hipStreamSynchronize(net->ctx->stream));
    return DL_OK;
  });
}

void dl_net_destroy(dl_net* net) {
  if (!net) return;
  (void)hipSetDevice(net->ctx->device);
  (void)hipStreamSynchronize(net->ctx->stream);
  delete net;
}

static int net_apply_prec(dl_net* net, dl_op* op, int prec, int nrhs, const double* B, double* Y, int mem) {
  return guard([&] {
    need(net && op, "NULL argument");
    need(prec == DL_FP32 || prec == DL_BF16, "prec must be DL_FP32 or DL_BF16");
    need(nrhs >= 0, "nrhs must be >= 0");
    if (nrhs == 0) return DL_OK;
    need(B && Y, "NULL argument");
    need(mem == DL_HOST || mem == DL_DEVICE, "mem must be DL_HOST or DL_DEVICE");
    check_net_op(net, op);
    use_device(op->ctx);
    DBuf<double2> bt = fields_in(op, B, nrhs, mem);
    DBuf<double2> yt((size_t)nrhs * op->lat.nc);
    net_apply(net, op, nrhs, bt.get(), yt.get(), prec == DL_BF16);
    fields_out(op, yt.get(), Y, nrhs, mem);
    return DL_OK;
  });
}

int dl_net_apply(dl_net* net, dl_op* op, int nrhs, const double* B, double* Y, int mem) {
  return net_apply_prec(net, op, DL_FP32, nrhs, B, Y, mem);
}

int dl_net_apply_prec(dl_net* net, dl_op* op, int prec, int nrhs, const double* B, double* Y, int mem) {
  return net_apply_prec(net, op, prec, nrhs, B, Y, mem);
}

int dl_net_set_projection(dl_net* net, const dl_eig* eig) {
  return guard([&] {
    need(net != nullptr, "net is NULL");
    need(!eig || eig->ctx == net->ctx, "eigenvector handle and network belong to different contexts");
    need(!eig || eig->kind == DL_MDAGM, "the projected training loss is the D-CG one (M^dag M eigenvectors)");
    net->proj = eig;
    return DL_OK;
  });
}

int dl_net_loss_grad(dl_net* net, dl_op* op, int n, const double* B, const double* X, int mem, double* loss,
                     double* grad) {
  return guard([&] {
    need(net && op && B && X && loss, "NULL argument");
    need(n >= 1, "need at least one pair");
    need(mem == DL_HOST || mem == DL_DEVICE, "mem must be DL_HOST or DL_DEVICE");
    check_net_op(net, op);
    use_device(op->ctx);
    DBuf<double2> bt = fields_in(op, B, n, mem);
    DBuf<double2> xt = fields_in(op, X, n, mem);
    *loss = net_loss_grad(net, op, n, bt.get(), xt.get(), grad != nullptr);
    if (grad) weights_to_host(net->G.get(), grad, op->ctx->stream);
    return DL_OK;
  });
}

int dl_net_train(dl_net* net, dl_op* op, int n, const double* B, const double* X, int mem, int batch, int steps,
                 double lr, double* losses) {
  return guard([&] {
    need(net && op && B && X, "NULL argument");
    need(n >= 1 && batch >= 1 && batch <= n, "need 1 <= batch <= n");
    need(steps >= 0, "steps must be >= 0");
    need(lr > 0 && std::isfinite(lr), "lr must be positive");
    need(mem == DL_HOST || mem == DL_DEVICE, "mem must be DL_HOST or DL_DEVICE");
    check_net_op(net, op);
    use_device(op->ctx);
    DBuf<double2> bt = fields_in(op, B, n, mem);
    DBuf<double2> xt = fields_in(op, X, n, mem);
    const int ngroups = n / batch;
    const long nc = op->lat.nc;
    for (int st = 0; st < steps; ++st) {
      const long g = st % ngroups;
      const double L = net_loss_grad(net, op, batch, bt.get() + g * batch * nc, xt.get() + g * batch * nc, true);
      if (losses) losses[st] = L;
      net_adam_step(net, (float)lr);
      if (verbose() && (st % 50 == 0 || st == steps - 1)) {
        std::fprintf(stderr, "[deflan] net train step %d/%d: loss %.5e\n", st, steps, L);
        std::fflush(stderr);
      }
    }
    DL_HIP(hipStreamSynchronize(op->ctx->stream));
    return DL_OK;
  });
}

int dl_eig_create(dl_op* op, int k, const double* V, int mem, dl_eig** out) {
  return guard([&] {
    need(op && out, "NULL argument");
    need(k >= 0 && k <= 512, "k must be in [0, 512]");
    need(k == 0 || V != nullptr, "V is NULL");
    use_device(op->ctx);
    DBuf<double2> Y = k ? fields_in(op, V, k, mem) : DBuf<double2>();
    *out = eig_build(op, k, std::move(Y), nullptr);
    return DL_OK;
  });
}

int dl_eig_info(const dl_eig* eig, int* k, double* evals, double* resid) {
  return guard([&] {
    need(eig != nullptr, "eig is NULL");
    if (k) *k = eig->k;
    if (evals) std::memcpy(evals, eig->evals.data(), eig->k * sizeof(double));
    if (resid) std::memcpy(resid, eig->resid.data(), eig->k * sizeof(double));
    return DL_OK;
  });
}

int dl_eig_vectors(const dl_eig* eig, double* V, int mem) {
  return guard([&] {
    need(eig && V, "NULL argument");
    need(mem == DL_HOST || mem == DL_DEVICE, "mem must be DL_HOST or DL_DEVICE");
    if (eig->k == 0) return DL_OK;
    use_device(eig->ctx);
    hipStream_t s = eig->ctx->stream;
    const Lattice& lat = eig->lat;
    const size_t bytes = (size_t)eig->k * lat.V * kSpin * sizeof(double2);
    if (mem == DL_DEVICE) {
      unpack_spinor(s, lat, eig->Y.get(), reinterpret_cast<double2*>(V), eig->k);
    } else {
      DBuf<double2> stage((size_t)eig->k * lat.V * kSpin);
      unpack_spinor(s, lat, eig->Y.get(), stage.get(), eig->k);
      DL_HIP(hipMemcpyAsync(V, stage.get(), bytes, hipMemcpyDeviceToHost, s));
      DL_HIP(hipStreamSynchronize(s));
    }
    DL_HIP(hipStreamSynchronize(s));
    return DL_OK;
  });
}

void dl_eig_destroy(dl_eig* eig) { delete eig; }

namespace {

// Handle file: a fixed header, then the host arrays, then the k eigenvectors in the caller's
// interleaved layout.  All numbers little-endian as in memory (the file is read back on the
// same kind of machine).
constexpr char kEigMagic[8] = {'D', 'L', 'E', 'I', 'G', '0', '0', '1'};
struct EigHeader {
  char magic[8];
  int32_t version, kind, k, dims[4], pad;
  double kappa;
  uint64_t fingerprint;
  int64_t V, zr_n, lamr_n;
};

struct File {
  FILE* f = nullptr;
  File(const char* path, const char* mode) : f(std::fopen(path, mode)) {}
  ~File() { if (f) std::fclose(f); }
};

void fwrite_all(FILE* f, const void* p, size_t bytes) {
  if (bytes && std::fwrite(p, 1, bytes, f) != bytes) fail(DL_E_INVALID, "write to the handle file failed");
}
void fread_all(FILE* f, void* p, size_t bytes) {
  if (bytes && std::fread(p, 1, bytes, f) != bytes) fail(DL_E_INVALID, "the handle file is truncated");
}

}  // namespace

int dl_eig_save(const dl_eig* eig, const char* path) {
  return guard([&] {
    need(eig && path, "NULL argument");
    use_device(eig->ctx);
    hipStream_t s = eig->ctx->stream;
    const Lattice& lat = eig->lat;
    EigHeader hd{};
    std::memcpy(hd.magic, kEigMagic, 8);
    hd.version = 1;
    hd.kind = eig->kind;
    hd.k = eig->k;
    for (int d = 0; d < 4; ++d) hd.dims[d] = lat.L[d];
    hd.kappa = eig->kappa;
    hd.fingerprint = eig->fingerprint;
    hd.V = lat.V;
    hd.zr_n = (int64_t)eig->Zr.n;
    hd.lamr_n = (int64_t)eig->lamr.n;
    std::vector<double> zr(eig->Zr.n), lamr(eig->lamr.n);
    if (!zr.empty()) DL_HIP(hipMemcpyAsync(zr.data(), eig->Zr.get(), zr.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    if (!lamr.empty())
      DL_HIP(hipMemcpyAsync(lamr.data(), eig->lamr.get(), lamr.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    DL_HIP(hipStreamSynchronize(s));
    File fh(path, "wb");
    if (!fh.f) fail(DL_E_INVALID, std::string("cannot open ") + path + " for writing");
    fwrite_all(fh.f, &hd, sizeof(hd));
    fwrite_all(fh.f, eig->evals.data(), eig->k * sizeof(double));
    fwrite_all(fh.f, eig->resid.data(), eig->k * sizeof(double));
    fwrite_all(fh.f, zr.data(), zr.size() * sizeof(double));
    fwrite_all(fh.f, lamr.data(), lamr.size() * sizeof(double));
    // one vector at a time through a staging field
    const size_t vbytes = (size_t)lat.V * kSpin * sizeof(double2);
    DBuf<double2> stage((size_t)lat.V * kSpin);
    std::vector<double2> host((size_t)lat.V * kSpin);
    for (int i = 0; i < eig->k; ++i) {
      unpack_spinor(s, lat, eig->Y.get() + (long)i * eig->nc, stage.get(), 1);
      DL_HIP(hipMemcpyAsync(host.data(), stage.get(), vbytes, hipMemcpyDeviceToHost, s));
      DL_HIP(hipStreamSynchronize(s));
      fwrite_all(fh.f, host.data(), vbytes);
    }
    if (std::fflush(fh.f) != 0) fail(DL_E_INVALID, "write to the handle file failed");
    return DL_OK;
  });
}

int dl_eig_load(dl_op* op, const char* path, dl_eig** out) {
  return guard([&] {
    need(op && path && out, "NULL argument");
    use_device(op->ctx);
    hipStream_t s = op->ctx->stream;
    const Lattice& lat = op->lat;
    File fh(path, "rb");
    if (!fh.f) fail(DL_E_INVALID, std::string("cannot open ") + path);
    EigHeader hd{};
    fread_all(fh.f, &hd, sizeof(hd));
    need(std::memcmp(hd.magic, kEigMagic, 8) == 0 && hd.version == 1, "not an eigenvector handle file");
    for (int d = 0; d < 4; ++d)
      if (hd.dims[d] != lat.L[d]) fail(DL_E_MISMATCH, "the handle file was saved for another lattice");
    if (hd.kind != op->kind || hd.kappa != op->kappa || hd.fingerprint != op->fingerprint)
      fail(DL_E_MISMATCH, "the handle file was saved for another operator (kind, kappa or links)");
    need(hd.k >= 0 && hd.k <= 512 && hd.V == lat.V, "corrupt handle header");
    const int k = hd.k;
    need(hd.zr_n == (k ? 4L * k * k : 0) && hd.lamr_n == (k ? 2L * k : 0), "corrupt handle header");
    std::vector<double> evals(k), resid(k), zr(hd.zr_n), lamr(hd.lamr_n);
    fread_all(fh.f, evals.data(), k * sizeof(double));
    fread_all(fh.f, resid.data(), k * sizeof(double));
    fread_all(fh.f, zr.data(), zr.size() * sizeof(double));
    fread_all(fh.f, lamr.data(), lamr.size() * sizeof(double));
    auto* e = new dl_eig();
    try {
      e->ctx = op->ctx;
      e->lat = lat;
      e->fingerprint = op->fingerprint;
      e->kappa = op->kappa;
      e->kind = op->kind;
      e->k = k;
      e->nc = lat.nc;
      e->evals = evals;
      e->resid = resid;
      if (k > 0) {
        e->Y.alloc((size_t)k * lat.nc);
        zero(s, (long)k * lat.nc, e->Y.get());  // padding sites
        const size_t vbytes = (size_t)lat.V * kSpin * sizeof(double2);
        DBuf<double2> stage((size_t)lat.V * kSpin);
        std::vector<double2> host((size_t)lat.V * kSpin);
        for (int i = 0; i < k; ++i) {
          fread_all(fh.f, host.data(), vbytes);
          DL_HIP(hipMemcpyAsync(stage.get(), host.data(), vbytes, hipMemcpyHostToDevice, s));
          pack_spinor(s, lat, stage.get(), e->Y.get() + (long)i * lat.nc, 1);
          DL_HIP(hipStreamSynchronize(s));
        }
        e->Zr.alloc(zr.size());
        e->lamr.alloc(lamr.size());
        DL_HIP(hipMemcpyAsync(e->Zr.get(), zr.data(), zr.size() * sizeof(double), hipMemcpyHostToDevice, s));
        DL_HIP(hipMemcpyAsync(e->lamr.get(), lamr.data(), lamr.size() * sizeof(double), hipMemcpyHostToDevice, s));
        DL_HIP(hipStreamSynchronize(s));
      }
      char extra;
      need(std::fread(&extra, 1, 1, fh.f) == 0, "the handle file has trailing data");
    } catch (...) {
      delete e;
      throw;
    }
    *out = e;
    return DL_OK;
  });
}

int dl_eig_lower(dl_op* op, dl_eig* eig, int prec, long* mvp) {
  return guard([&] {
    need(op && eig, "NULL argument");
    need(prec == DL_FP64 || prec == DL_FP32 || prec == DL_BF16, "prec must be DL_FP64, DL_FP32 or DL_BF16");
    if (eig->fingerprint != op->fingerprint || eig->kind != op->kind)
      fail(DL_E_MISMATCH, "eigenvector handle was built for a different operator");
    use_device(op->ctx);
    const long used = eig_lower(op, eig, prec);
    if (mvp) *mvp = used;
    return DL_OK;
  });
}

int dl_tsk_project(dl_ctx* ctx, long n, int nv, const double* V, double* w, double* c, int subtract, int mem) {
  return guard([&] {
    need(ctx && V && w && c, "NULL argument");
    need(n > 0 && nv > 0 && nv <= 512, "need n > 0 and 0 < nv <= 512");
    need(mem == DL_HOST || mem == DL_DEVICE, "mem must be DL_HOST or DL_DEVICE");
    use_device(ctx);
    hipStream_t s = ctx->stream;
    DBuf<double2> Vd, wd, cd(nv);
    const double2 *vp = reinterpret_cast<const double2*>(V);
    double2* wp = reinterpret_cast<double2*>(w);
    double2* cp = reinterpret_cast<double2*>(c);
    if (mem == DL_HOST) {
      Vd.alloc((size_t)nv * n);
      wd.alloc(n);
      DL_HIP(hipMemcpyAsync(Vd.get(), V, (size_t)nv * n * sizeof(double2), hipMemcpyHostToDevice, s));
      DL_HIP(hipMemcpyAsync(wd.get(), w, (size_t)n * sizeof(double2), hipMemcpyHostToDevice, s));
      vp = Vd.get();
      wp = wd.get();
      cp = cd.get();
    }
    DBuf<double> part((size_t)2 * nv * tsk_nblocks(n));
    int nb;
    {
      TimeScope ts(ctx, T_TSK_DOTS);
      nb = tsk_dots(s, n, nv, vp, n, nullptr, wp, part.get());
    }
    sum_partials(s, part.get(), nb, 2 * nv, reinterpret_cast<double*>(cp));
    if (subtract) {
      TimeScope ts(ctx, T_TSK_UPDATE);
      tsk_update(s, n, nv, vp, n, nullptr, cp, -1.0, wp);
    }
    if (mem == DL_HOST) {
      DL_HIP(hipMemcpyAsync(c, cp, (size_t)nv * sizeof(double2), hipMemcpyDeviceToHost, s));
      if (subtract) DL_HIP(hipMemcpyAsync(w, wp, (size_t)n * sizeof(double2), hipMemcpyDeviceToHost, s));
    }
    DL_HIP(hipStreamSynchronize(s));
    return DL_OK;
  });
}

int dl_tsk_project_noalloc(dl_ctx* ctx, long n, int nv, const double* V, double* w, double* c, int subtract) {
  return guard([&] {
    need(ctx && V && w && c, "NULL argument");
    need(n > 0 && nv > 0 && nv <= 512, "need n > 0 and 0 < nv <= 512");
    use_device(ctx);
    tsk_project_noalloc(ctx, n, nv, reinterpret_cast<const double2*>(V), reinterpret_cast<double2*>(w),
                        reinterpret_cast<double2*>(c), subtract);
    DL_HIP(hipStreamSynchronize(ctx->stream));
    return DL_OK;
  });
}

int dl_tsk_project_multi(dl_ctx* ctx, long n, int nv, const double* V, int nw, const double* W, double* C, double* X,
                         int mem) {
  return guard([&] {
    need(ctx && V && W && C, "NULL argument");
    need(n > 0 && nv > 0 && nv <= 512, "need n > 0 and 0 < nv <= 512");
    need(nw >= 1 && nw <= 16, "need 1 <= nw <= 16");
    need(mem == DL_HOST || mem == DL_DEVICE, "mem must be DL_HOST or DL_DEVICE");
    use_device(ctx);
    hipStream_t s = ctx->stream;
    DBuf<double2> Vd, Wd, Xd, Cd;
    const double2* vp = reinterpret_cast<const double2*>(V);
    const double2* wp = reinterpret_cast<const double2*>(W);
    double2* xp = reinterpret_cast<double2*>(X);
    double2* cp = reinterpret_cast<double2*>(C);
    if (mem == DL_HOST) {
      Vd.alloc((size_t)nv * n);
      Wd.alloc((size_t)nw * n);
      Cd.alloc((size_t)nw * nv);
      DL_HIP(hipMemcpyAsync(Vd.get(), V, (size_t)nv * n * sizeof(double2), hipMemcpyHostToDevice, s));
      DL_HIP(hipMemcpyAsync(Wd.get(), W, (size_t)nw * n * sizeof(double2), hipMemcpyHostToDevice, s));
      vp = Vd.get();
      wp = Wd.get();
      cp = Cd.get();
      if (X) {
        Xd.alloc((size_t)nw * n);
        DL_HIP(hipMemcpyAsync(Xd.get(), X, (size_t)nw * n * sizeof(double2), hipMemcpyHostToDevice, s));
        xp = Xd.get();
      }
    }
    constexpr int kRows = 64;
    DBuf<double> part((size_t)2 * kRows * nw * tsk_multi_nblocks(n));
    for (int j0 = 0; j0 < nv; j0 += kRows) {
      const int m = std::min(kRows, nv - j0);
      int np;
      {
        TimeScope ts(ctx, T_TSK_DOTS);
        np = tsk_dots_multi(s, n, m, vp + (long)j0 * n, n, wp, n, nw, nullptr, part.get());
      }
      for (int r = 0; r < nw; ++r)
        sum_partials(s, part.get() + (size_t)2 * r * m * np, np, 2 * m, reinterpret_cast<double*>(cp + (long)r * nv + j0));
    }
    if (X) {
      TimeScope ts(ctx, T_TSK_UPDATE);
      tsk_update_multi(s, n, nv, vp, n, cp, nw, nullptr, xp, n);
    }
    if (mem == DL_HOST) {
      DL_HIP(hipMemcpyAsync(C, cp, (size_t)nw * nv * sizeof(double2), hipMemcpyDeviceToHost, s));
      if (X) DL_HIP(hipMemcpyAsync(X, xp, (size_t)nw * n * sizeof(double2), hipMemcpyDeviceToHost, s));
    }
    DL_HIP(hipStreamSynchronize(s));
    return DL_OK;
  });
}

int dl_tsk_project_lowp(dl_ctx* ctx, int prec, long n, int nv, const double* V, int nw, const double* W, double* C,
                        double* X, int mem) {
  return guard([&] {
    need(ctx && V && W && C, "NULL argument");
    need(prec == DL_FP32 || prec == DL_BF16, "prec must be DL_FP32 or DL_BF16");
    need(n > 0 && nv > 0 && nv <= 512, "need n > 0 and 0 < nv <= 512");
    need(nw >= 1 && nw <= 16, "need 1 <= nw <= 16");
    need(mem == DL_HOST || mem == DL_DEVICE, "mem must be DL_HOST or DL_DEVICE");
    use_device(ctx);
    hipStream_t s = ctx->stream;
    DBuf<double2> Vd, Wd, Xd, Cd;
    const double2* vp = reinterpret_cast<const double2*>(V);
    const double2* wp = reinterpret_cast<const double2*>(W);
    double2* xp = reinterpret_cast<double2*>(X);
    double2* cp = reinterpret_cast<double2*>(C);
    if (mem == DL_HOST) {
      Vd.alloc((size_t)nv * n);
      Wd.alloc((size_t)nw * n);
      Cd.alloc((size_t)nw * nv);
      DL_HIP(hipMemcpyAsync(Vd.get(), V, (size_t)nv * n * sizeof(double2), hipMemcpyHostToDevice, s));
      DL_HIP(hipMemcpyAsync(Wd.get(), W, (size_t)nw * n * sizeof(double2), hipMemcpyHostToDevice, s));
      vp = Vd.get();
      wp = Wd.get();
      cp = Cd.get();
      if (X) {
        Xd.alloc((size_t)nw * n);
        DL_HIP(hipMemcpyAsync(Xd.get(), X, (size_t)nw * n * sizeof(double2), hipMemcpyHostToDevice, s));
        xp = Xd.get();
      }
    }
    // rounded copies at a stride that keeps every field 16-byte aligned
    const long ld = (n + 3) / 4 * 4;
    DBuf<float2> v32((size_t)nv * ld), w32, x32;
    DBuf<bf2> v16, w16;
    for (int j = 0; j < nv; ++j) round_f32(s, n, vp + (long)j * n, v32.get() + (long)j * ld);
    if (prec == DL_BF16) {
      v16.alloc((size_t)nv * ld);
      w16.alloc((size_t)nw * ld);
      for (int j = 0; j < nv; ++j) round_bf16(s, n, vp + (long)j * n, v16.get() + (long)j * ld);
      for (int r = 0; r < nw; ++r) round_bf16(s, n, wp + (long)r * n, w16.get() + (long)r * ld);
    } else {
      w32.alloc((size_t)nw * ld);
      for (int r = 0; r < nw; ++r) round_f32(s, n, wp + (long)r * n, w32.get() + (long)r * ld);
    }
    constexpr int kRows = 128;
    DBuf<double> part((size_t)2 * kRows * nw * tsk_lowp_nblocks(n, prec));
    for (int j0 = 0; j0 < nv; j0 += kRows) {
      const int m = std::min(kRows, nv - j0);
      int np;
      {
        TimeScope ts(ctx, T_TSK_DOTS);
        np = prec == DL_BF16
                 ? tsk_dots_lowp(s, n, m, v16.get() + (long)j0 * ld, ld, w16.get(), ld, nw, nullptr, part.get())
                 : tsk_dots_lowp(s, n, m, v32.get() + (long)j0 * ld, ld, w32.get(), ld, nw, nullptr, part.get());
      }
      for (int r = 0; r < nw; ++r)
        sum_partials(s, part.get() + (size_t)2 * r * m * np, np, 2 * m,
                     reinterpret_cast<double*>(cp + (long)r * nv + j0));
    }
    if (X) {
      TimeScope ts(ctx, T_TSK_UPDATE);
      tsk_update_multi32(s, n, nv, v32.get(), ld, cp, nw, nullptr, xp, n);
    }
    if (mem == DL_HOST) {
      DL_HIP(hipMemcpyAsync(C, cp, (size_t)nw * nv * sizeof(double2), hipMemcpyDeviceToHost, s));
      if (X) DL_HIP(hipMemcpyAsync(X, xp, (size_t)nw * n * sizeof(double2), hipMemcpyDeviceToHost, s));
    }
    DL_HIP(hipStreamSynchronize(s));
    return DL_OK;
  });
}

int dl_tsk_combine(dl_ctx* ctx, long n, int nv, const double* V, const double* G, int ny, double* Y, int mem) {
  return guard([&] {
    need(ctx && V && G && Y, "NULL argument");
    need(n > 0 && nv > 0 && nv <= 512 && ny > 0, "need n > 0, 0 < nv <= 512, ny > 0");
    need(mem == DL_HOST || mem == DL_DEVICE, "mem must be DL_HOST or DL_DEVICE");
    use_device(ctx);
    hipStream_t s = ctx->stream;
    DBuf<double2> Vd, Yd;
    DBuf<double> Gd((size_t)nv * ny);
    const double2* vp = reinterpret_cast<const double2*>(V);
    double2* yp = reinterpret_cast<double2*>(Y);
    if (mem == DL_HOST) {
      Vd.alloc((size_t)nv * n);
      Yd.alloc((size_t)ny * n);
      DL_HIP(hipMemcpyAsync(Vd.get(), V, (size_t)nv * n * sizeof(double2), hipMemcpyHostToDevice, s));
      vp = Vd.get();
      yp = Yd.get();
      DL_HIP(hipMemcpyAsync(Gd.get(), G, (size_t)nv * ny * sizeof(double), hipMemcpyHostToDevice, s));
    } else {
      DL_HIP(hipMemcpyAsync(Gd.get(), G, (size_t)nv * ny * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    {
      TimeScope ts(ctx, T_TSK_UPDATE);
      tsk_combine(s, n, nv, vp, n, nullptr, Gd.get(), ny, ny, yp, n, nullptr, 0);
    }
    if (mem == DL_HOST)
      DL_HIP(hipMemcpyAsync(Y, yp, (size_t)ny * n * sizeof(double2), hipMemcpyDeviceToHost, s));
    DL_HIP(hipStreamSynchronize(s));
    return DL_OK;
  });
}

int dl_small_eigh(dl_ctx* ctx, int n, const double* A, double* evals, double* Z) {
  return guard([&] {
    need(ctx && A && evals && Z, "NULL argument");
    need(n >= 1 && n <= 512, "n must be in [1, 512]");
    use_device(ctx);
    hipStream_t s = ctx->stream;
    DBuf<double> Ad((size_t)n * n), Zd((size_t)n * n), ev(n), work(small_eigh_work(n));
    DL_HIP(hipMemcpyAsync(Ad.get(), A, (size_t)n * n * sizeof(double), hipMemcpyHostToDevice, s));
    {
      TimeScope ts(ctx, T_SMALL);
      small_eigh(s, n, Ad.get(), Zd.get(), ev.get(), work.get());
    }
    DL_HIP(hipMemcpyAsync(evals, ev.get(), n * sizeof(double), hipMemcpyDeviceToHost, s));
    DL_HIP(hipMemcpyAsync(Z, Zd.get(), (size_t)n * n * sizeof(double), hipMemcpyDeviceToHost, s));
    DL_HIP(hipStreamSynchronize(s));
    return DL_OK;
  });
}

}  // extern "C"
