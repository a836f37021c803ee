// Internal declarations shared by the HIP translation units of libdeflan.
//
// Device layout of a lattice field (spinor or links) is site-major and tiled:
// sites are grouped in tiles of 64 consecutive sites (one wavefront), and
// inside a tile the complex components are outermost, so that component c of
// the 64 sites of a tile is one contiguous 1 KiB run (FP64):
//
//     spinor:  elem(site, c) = ((site / 64) * 12 + c) * 64 + site % 64,  c = spin*3 + colour
//     links:   elem(site, mu, a, b) = ((site / 64) * 36 + mu*9 + a*3 + b) * 64 + site % 64
//
// A wavefront reading one component of 64 consecutive sites issues one fully
// coalesced 16-byte-per-lane load.  Padding sites of the last tile are zero and
// stay zero under every kernel, so reductions over the padded length equal
// reductions over the lattice.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/deflan.h"

namespace dl {

// BF16 complex storage: the upper halves of the two FP32 parts (round to nearest even).
struct __align__(4) bf2 {
  unsigned short x, y;
};

// complex element type of a real type: double -> double2, float -> float2
template <class R>
using cplx_t = typename std::conditional<sizeof(R) == 8, double2, float2>::type;

constexpr int kTile = 64;      // sites per tile (= wavefront size)
constexpr int kSpin = 12;      // complex components per spinor site
constexpr int kLinkC = 36;     // complex components per site of links (4 x 3 x 3)
constexpr int kBlock = 256;    // threads per block of the streaming kernels
constexpr int kMaxPartials = 16384;  // upper bound of blocks writing one reduction column

struct Error {
  int code;
  std::string msg;
};

void set_error(const std::string& msg);
[[noreturn]] void fail(int code, const std::string& msg);
void hip_check(hipError_t e, const char* what, const char* file, int line);
#define DL_HIP(x) ::dl::hip_check((x), #x, __FILE__, __LINE__)

struct Lattice {
  int L[4];        // Lx, Ly, Lz, Lt
  long V;          // sites of a field (eo: the sites of one parity, half the lattice)
  long ntiles;     // ceil(V / 64)
  long nc;         // complex elements of a padded spinor field = ntiles * 64 * 12
  long nl;         // complex elements of the padded links of the whole lattice
  int eo = 0;      // 1: fields hold the even sites only (the even-odd Schur operator)
};

Lattice make_lattice(const int dims[4]);
// The even half of the lattice of dims (every extent even): fields of V/2 sites in increasing
// full-site order, half index = full site / 2 (tiled like a full field); links stay full.
Lattice make_lattice_eo(const int dims[4]);

// ---- device memory --------------------------------------------------------
void* dmalloc(size_t bytes);  // cached per device (freed blocks are reused by size)
void dfree(void* p);
void dmem_trim(int dev);      // release the device's cached blocks

template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  explicit DBuf(size_t count) { alloc(count); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DBuf() { release(); }
  // Contents are undefined: kernels write every element before reading it, and
  // buffers that must start at zero are cleared on the context's stream.
  void alloc(size_t count) {
    release();
    if (count) p = static_cast<T*>(dmalloc(count * sizeof(T)));
    n = count;
  }
  void release() { if (p) dfree(p); p = nullptr; n = 0; }
  T* get() const { return p; }
};

// ---- kernel timing --------------------------------------------------------
// T_WILSON: stencils with FP32 or BF16 spinors; T_WILSON64: FP64 stencils.
enum TimerId { T_WILSON = 0, T_TSK_DOTS, T_TSK_UPDATE, T_SMALL, T_WILSON64, T_COUNT };

struct Timers {
  bool enabled = false;
  struct Pair { hipEvent_t a, b; int id; double bytes; };
  std::vector<Pair> pending;
  std::vector<hipEvent_t> pool;
  long launches[T_COUNT] = {0};
  double ms[T_COUNT] = {0};
  double bytes[T_COUNT] = {0};  // algorithmic bytes moved by the timed launches
  hipEvent_t take();
  void begin(hipStream_t s, int id, hipEvent_t* a);
  void end(hipStream_t s, int id, hipEvent_t a, double bytes);
  void collect();  // sync pending events and accumulate
  void reset();
  ~Timers();
};

}  // namespace dl

struct dl_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  dl::Timers timers;
  // scratch used by reductions: partial sums and a pinned host mirror
  dl::DBuf<double> partials;   // kMaxPartials * 2 * 512 doubles
  double* pinned = nullptr;    // 4096 doubles of pinned host memory
};

namespace dl {

// RAII scope that brackets kernel launches with timing events when enabled.
struct TimeScope {
  dl_ctx* ctx;
  int id;
  double bytes;
  hipEvent_t a = nullptr;
  TimeScope(dl_ctx* c, int i, double algorithmic_bytes = 0.0) : ctx(c), id(i), bytes(algorithmic_bytes) {
    if (ctx->timers.enabled) ctx->timers.begin(ctx->stream, id, &a);
  }
  ~TimeScope() {
    if (ctx->timers.enabled && a) ctx->timers.end(ctx->stream, id, a, bytes);
  }
};

// ---- launchers: layout ------------------------------------------------------
void pack_spinor(hipStream_t s, const Lattice& lat, const double2* host_layout, double2* tiled, int nfield);
void unpack_spinor(hipStream_t s, const Lattice& lat, const double2* tiled, double2* host_layout, int nfield);
void pack_links(hipStream_t s, const Lattice& lat, const double2* host_layout, double2* tiled);

// ---- launchers: Wilson operator ------------------------------------------------
// Launch shape of the stencil: variant 0-3 = one thread per site with (threads per block,
// occupancy hint) among {(256,2), (128,2), (512,1), (256,1)}; 4-6 = one thread per (x,y,z)
// site marching through time chunks of 4, 8, 16 slices; 7-10 = the marching form with 64
// sites per block, links staged in LDS and shared by (rhs per block, T) = (4, 8), (4, 16),
// (8, 8), (2, 8); 11-14 = the marching form with each slice's spinors staged in LDS (11: with
// the x, y links too, FP32 only; T = 8, 8, 16, 8; 14 issues each hop's loads one hop ahead); order = block order (0: rhs fastest, XCD-contiguous; 1: sites
// fastest, XCD-contiguous; 2: rhs fastest, hardware order).  Chosen by the autotuner.
// 15-17 = one thread per site for 2 or 4 rhs of a group (256 threads; 2 rhs with 128 threads), each
// hop's link loaded once for the group.  18-19 = the slice-staged form with each block a box of
// whole x rows spanning y and z (T = 8, 16), so z neighbours inside the box come from LDS too
// (variants 12 and 13 where no box tiles the slice).
constexpr int kWilsonVariants = 20;
constexpr int kWilsonOrders = 3;
struct WilsonCfg {
  int variant = 0;
  int order = 0;
};
// which: 0 M, 1 M^dag, 2 gamma5 M.  red: 0 none, 1 ||out||^2 partials, 2 Re<in,out> partials.
// Returns the number of partials per rhs written to `part` (0 if red == 0).
int wilson_f64(hipStream_t s, const Lattice& lat, const double2* U, double kappa, int which,
               const double2* in, double2* out, int red, double* part, WilsonCfg cfg = WilsonCfg());
void gamma5_f64(hipStream_t s, const Lattice& lat, const double2* in, double2* out);
// Even-odd operator (lat.eo): op = Mhat = 1 - kappa^2 D_eo D_oe on the even half fields (which 0),
// Mhat^dag (1), gamma5 Mhat (2), through an odd intermediate field in the arithmetic precision
// held in a per-stream scratch buffer (eo_reserve grows it ahead of graph capture).
void eo_reserve(hipStream_t s, size_t bytes);
void eo_release(hipStream_t s);
// Full fields (tiled, whole lattice `full`) <-> half fields (tiled, lat.eo) of parity par.
void eo_split(hipStream_t s, const Lattice& full, const double2* in, double2* half, int par, int nfield);
void eo_merge(hipStream_t s, const Lattice& full, const double2* half, double2* out, int par, int nfield);
// out_{par} = kappa_fac * D_{par, 1-par} in_{1-par} + add_{par} (FP64 half fields; add may be NULL).
void eo_hop_f64(hipStream_t s, const Lattice& lat, const double2* U, double kappa_fac, int par, const double2* in,
                const double2* add, double2* out);
// Batched Wilson apply in FP64 (R = double) or FP32 (R = float): nrhs fields at stride fstride.
// Partials (red != 0) are column-major [nrhs][wilson_nbs(lat)].  Returns wilson_nbs(lat) or 0.
int wilson_nbs(const Lattice& lat, const WilsonCfg& cfg);
int wilson_max_nbs(const Lattice& lat);  // partials per rhs of the widest-grid variant
// SV: spinor storage (double2 with R = double; float2 or bf2 with R = float); arithmetic in R.
template <class R, class SV>
int wilson_batched(hipStream_t s, const Lattice& lat, const cplx_t<R>* U, double kappa, int which,
                   const SV* in, SV* out, long fstride, int nrhs, int red, const double* scale,
                   const int* active, double* part, WilsonCfg cfg = WilsonCfg());

// r = b - M x in FP64 for nrhs whole-lattice fields at stride fstride, with ||r||^2 partials
// column-major [nrhs][nbs] (an inactive rhs: r untouched, partials 0); returns nbs.  The
// time-marching stencil computes it in its epilogue, so M x is never stored.  With lo (and
// r == nullptr) the residual is stored only rounded to lo_prec (DL_FP32: float2, DL_BF16: bf2,
// through FP32) at the same offsets, and the partials sum the squares of the stored values.
int wilson_residual_f64(hipStream_t s, const Lattice& lat, const double2* U, double kappa, const double2* x,
                        const double2* b, double2* r, long fstride, int nrhs, const int* active, double* part,
                        void* lo = nullptr, int lo_prec = 0);

// Several lattices in one stencil launch (the multi-lattice batched solver): one item per
// operator, right-hand sides [rhs0, rhs0 + nrhs) of the batch, nbs = ceil(V / 256) site blocks,
// blocks [block0, block0 + nbs * nrhs) of the launch.  Field j of the batch starts at offs[j].
struct WilsonItem {
  const void* U;   // links of the item's precision (double2 or float2), tiled
  double kappa;
  int L[4];
  long V, Vpad;
  int rhs0, nrhs, nbs, block0;
};
// Partials (red != 0) are column-major [rhs][pstride], pstride >= every item's nbs.
template <class R, class SV>
void wilson_multi(hipStream_t s, const WilsonItem* d_items, int nitems, int nblocks, int pstride, int which,
                  const SV* in, SV* out, const long* offs, int red, const double* scale, const int* active,
                  double* part);

// ---- launchers: BLAS-1 ------------------------------------------------------
int nblocks_for(long n);  // partial count used by the streaming reductions for length n
// partial sums
int dot_partials(hipStream_t s, long n, const double2* a, const double2* b, double* part);  // complex, 2 per block
int norm2_partials(hipStream_t s, long n, const double2* a, double* part);                  // 1 per block
// Partials are stored column-major: part[col * nparts + block].
// out[col] = sum_i part[col * nparts + i] (fixed order); grid = width blocks
void sum_partials(hipStream_t s, const double* part, int nparts, int width, double* out);

void copy(hipStream_t s, long n, const double2* a, double2* b);
void zero(hipStream_t s, long n, double2* a);
void round_f32(hipStream_t s, long n, const double2* a, float2* b);  // b = (float) a
void widen_f64(hipStream_t s, long n, const float2* a, double2* b);  // b = (double) a
void round_bf16(hipStream_t s, long n, const double2* a, bf2* b);    // b = bf16(float(a)), nearest even
// Position-dependent 64-bit hash of n complex numbers (bit patterns): the wrap-around sum of a
// mixed (index, bits) word per element, so it is independent of the summation order and any
// single changed element changes it (up to 64-bit collisions).  Synchronises the stream.
uint64_t field_hash(hipStream_t s, long n, const double2* a);

// ---- the no-allocation projection (noalloc.hip) ------------------------------------
void noalloc_init(int device);  // once per device, with the device current (context creation)
void widen_bf16(hipStream_t s, long n, const bf2* a, double2* b);    // b = (double) a

}  // namespace dl
