// C ABI of libpnof: context, validation, workspace planning and the per-call drivers.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "pnof.h"

using namespace pnof;

// Workspace of pnof_lagrangian_noalloc: one static array per GPU, held until the process ends.  In
// host code `scratch` is only a stand-in for the symbol; its device address on each GPU comes from
// hipGetSymbolAddress (taken once per device by pnof_create) and only that address is used.
static __device__ __align__(256) char scratch[PNOF_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};
}  // namespace

struct pnof_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  rocblas_handle blas = nullptr;
  std::string err;
  char* ext_ws = nullptr;
  size_t ext_bytes = 0;
  char* own_ws = nullptr;
  size_t own_bytes = 0;
  pnof_tuning tune{0, 0, 0, 0, 0};
  int* host_info = nullptr;  // pinned
  // second stream (default priority) for work that overlaps the main stream's, forked and joined
  // with events; created on first use
  hipStream_t aux = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  hipEvent_t pipe_ev[4] = {nullptr, nullptr, nullptr, nullptr};   // chunk pipeline of the split path
  // measurement: launches of the contraction kernels bracketed by events on the stream
  bool profiling = false;
  struct Ev { int stage; hipEvent_t a, b; };
  std::vector<Ev> evs;
  std::vector<hipEvent_t> pool;
  // buffers of the driver calls (occupation and orbital optimisation, NOF-MP2 terms), kept from one
  // call to the next and grown on demand, so that repeated calls allocate nothing
  struct Slot { void* p; size_t bytes; };
  std::vector<Slot> slots;
  size_t slot_top = 0;
  // integrals bound by pnof_bind_integrals: their per-chunk row bounds (split mode) and the key they
  // were computed under
  struct Bound {
    const void* ints = nullptr;
    int nbf = 0, naux = 0, kind = 0, pc = 0;
    uint32_t* words = nullptr;   // 2 per chunk (device)
    size_t nwords = 0, cap = 0;
  } bound;
};

namespace {

thread_local std::string g_err;

pnof_status fail(pnof_ctx ctx, pnof_status st, const std::string& msg) {
  g_err = msg;
  if (ctx) ctx->err = msg;
  return st;
}

#define DEV_CHECK(ctx, expr)                                                                  \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(ctx, PNOF_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

// Bump allocator over a workspace region; with base == nullptr it only measures.
struct Arena {
  char* base;
  size_t off = 0;
  explicit Arena(char* b) : base(b) {}
  template <typename T>
  T* take(long long count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * (size_t)(count > 0 ? count : 0);
    return p;
  }
};

// The context's second stream (default priority) and the events that fork and join it.
pnof_status ensure_aux(pnof_ctx ctx) {
  if (!ctx->aux) DEV_CHECK(ctx, hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
  if (!ctx->fork_ev) DEV_CHECK(ctx, hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
  if (!ctx->join_ev) DEV_CHECK(ctx, hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming));
  for (hipEvent_t& e : ctx->pipe_ev)
    if (!e) DEV_CHECK(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return PNOF_OK;
}

// Joins the context's second stream into its stream when a scope that forked it ends (on every
// return path, so that no work of the call is left running on the second stream).
struct AuxJoin {
  pnof_ctx ctx;
  bool forked = false;
  explicit AuxJoin(pnof_ctx c) : ctx(c) {}
  ~AuxJoin() {
    if (!forked) return;
    if (hipEventRecord(ctx->join_ev, ctx->aux) == hipSuccess) hipStreamWaitEvent(ctx->stream, ctx->join_ev, 0);
  }
};

#define RB_CHECK(expr)                    \
  do {                                    \
    const pnof_status st_ = (expr);       \
    if (st_ != PNOF_OK) return st_;       \
  } while (0)

hipEvent_t pool_event(pnof_ctx ctx) {
  if (!ctx->pool.empty()) {
    hipEvent_t e = ctx->pool.back();
    ctx->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch with events when the context is profiling.
struct StageTimer {
  pnof_ctx ctx;
  int stage;
  hipEvent_t a = nullptr;
  StageTimer(pnof_ctx c, int st) : ctx(c), stage(st) {
    if (ctx->profiling && (a = pool_event(ctx))) hipEventRecord(a, ctx->stream);
  }
  ~StageTimer() {
    if (!a) return;
    hipEvent_t b = pool_event(ctx);
    if (!b) return;
    hipEventRecord(b, ctx->stream);
    ctx->evs.push_back({stage, a, b});
  }
};
#define TIMED(ctx, stage, expr) [&]() { StageTimer t_(ctx, stage); return (expr); }()

bool is_df(int ints) { return ints == PNOF_INTS_DF_F64 || ints == PNOF_INTS_DF_BF16; }

pnof_status check_problem(pnof_ctx ctx, const pnof_problem* p) {
  if (!p) return fail(ctx, PNOF_E_ARG, "problem is NULL");
  if (p->nbf <= 0) return fail(ctx, PNOF_E_SHAPE, "nbf must be positive");
  if (p->npairs <= 0 || p->ncwo <= 0) return fail(ctx, PNOF_E_SHAPE, "npairs and ncwo must be positive");
  if (p->nsingle < 0) return fail(ctx, PNOF_E_SHAPE, "nsingle must not be negative");
  const long long nact = (long long)p->npairs * (p->ncwo + 1) + p->nsingle;
  if (nact > p->nbf) return fail(ctx, PNOF_E_SHAPE, "npairs*(ncwo+1) exceeds nbf");
  if (p->functional != PNOF5 && p->functional != PNOF7 && p->functional != PNOF7S)
    return fail(ctx, PNOF_E_ARG, "unknown functional");
  if (p->precision != PNOF_FP64 && p->precision != PNOF_FP32 && p->precision != PNOF_BF16 &&
      p->precision != PNOF_BF16_SPLIT)
    return fail(ctx, PNOF_E_ARG, "unknown precision");
  if (p->ints != PNOF_INTS_ERI4_F64 && !is_df(p->ints)) return fail(ctx, PNOF_E_ARG, "unknown integral kind");
  if (p->flags & ~PNOF_CHECK_FINITE) return fail(ctx, PNOF_E_ARG, "unknown flag bits");
  if (p->ints == PNOF_INTS_ERI4_F64) {
    if (p->naux != 0) return fail(ctx, PNOF_E_SHAPE, "naux must be 0 with explicit four-index integrals");
    if (p->nbf > 64) return fail(ctx, PNOF_E_SHAPE, "explicit four-index integrals need nbf <= 64");
    if (p->precision != PNOF_FP64) return fail(ctx, PNOF_E_DTYPE, "explicit integrals are float64 only");
  } else {
    if (p->naux <= 0) return fail(ctx, PNOF_E_SHAPE, "naux must be positive for density fitting");
  }
  if ((long long)p->nbf * p->nbf > (1LL << 31)) return fail(ctx, PNOF_E_SHAPE, "nbf too large");
  return PNOF_OK;
}

// ------------------------------------------------------------------------ planning
struct Plan {
  int nbf, nact, naux, npairs, ncwo, nsingle, functional, prec, ints;
  int pc, ns2, ns3, xv, yv;
  int ldk, ldx, ldxx, ldw, nact32;
  bool split;   // bf16 family
  bool f32;     // PNOF_FP32: the float64 path's kernels in float32
  int terms;    // 1 or 3
};

Plan make_plan(const pnof_problem* p, const pnof_tuning& tu) {
  Plan pl{};
  pl.nbf = p->nbf;
  pl.nact = p->npairs * (p->ncwo + 1) + p->nsingle;
  pl.nsingle = p->nsingle;
  pl.naux = p->naux;
  pl.npairs = p->npairs;
  pl.ncwo = p->ncwo;
  pl.functional = p->functional;
  pl.prec = p->precision;
  pl.ints = p->ints;
  pl.split = (p->precision == PNOF_BF16 || p->precision == PNOF_BF16_SPLIT);
  pl.f32 = (p->precision == PNOF_FP32);
  pl.terms = p->precision == PNOF_BF16_SPLIT ? 3 : 1;
  const int tile = pl.split ? 128 : 64;
  // workspace rows padded to multiples of 32 (zero pads): whole k-tiles never need masking
  pl.ldk = (int)round_up(pl.nbf, 32);
  pl.ldx = (int)round_up(pl.nbf, 32);
  pl.ldxx = (int)round_up(pl.nact, 32);
  pl.ldw = (int)round_up(pl.nact, 32);
  pl.nact32 = (int)round_up(pl.nact, 32);
  if (!is_df(p->ints)) { pl.pc = pl.ns2 = pl.ns3 = 1; pl.xv = pl.yv = 1; return pl; }
  // block tiles of the split contractions: the 256 x 256 tile (variant 3) halves the LDS and operand
  // traffic per product, and is the automatic choice when it pads the output no more than the 128
  // tiling does (within 5 %) and both extents reach 512
  auto pick = [&](int req, int m, int n) {
    if (!pl.split) return 1;
    if (req > 0) return req;
    const double a128 = (double)round_up(m, 128) * round_up(n, 128), a256 = (double)round_up(m, 256) * round_up(n, 256);
    return (m >= 512 && n >= 512 && a256 <= 1.05 * a128) ? 3 : 1;
  };
  pl.xv = pick(tu.x_variant, pl.nact, pl.nbf);
  pl.yv = pick(tu.y_variant, pl.nbf, pl.nact);
  const int xm = pl.xv == 3 ? 256 : tile, xn = pl.xv >= 2 ? 256 : tile;
  const int ym = pl.yv >= 2 ? 256 : tile, yn = pl.yv == 3 ? 256 : tile;
  const long long t1 = (long long)cdiv(pl.nact, xm) * cdiv(pl.nbf, xn);
  // enough blocks per launch to fill the chip, and enough rows per chunk that the per-split K
  // partials (ns2 x nact^2, read-modified-written once per chunk) stay small next to X and W
  long long pc = tu.pchunk > 0 ? tu.pchunk : std::max(64LL, (4096 + t1 - 1) / t1);
  const long long per_p = pl.split ? (long long)(2LL * pl.nact32 * pl.ldx + 2LL * pl.nact32 * pl.ldw) * 2 +
                                         (p->ints == PNOF_INTS_DF_F64 ? 4LL * pl.nbf * pl.nbf : 0)
                                   : pl.f32 ? (long long)(pl.nact * pl.ldx + pl.nact * pl.ldw) * 4
                                            : (long long)(pl.nact * pl.ldx + pl.nact * pl.ldw) * 8 +
                                                  (p->ints == PNOF_INTS_DF_BF16 ? 8LL * pl.nbf * pl.nbf : 0);
  const long long cap = std::max(1LL, (2LL << 30) / std::max(1LL, per_p));
  if (tu.pchunk <= 0) pc = std::min(pc, cap);
  pc = std::min<long long>(pc, pl.naux);
  pl.pc = (int)std::max(1LL, pc);
  const int tt = cdiv(pl.nact, tile);
  const long long ntri = (long long)tt * (tt + 1) / 2;
  pl.ns2 = tu.nsplit_b > 0 ? tu.nsplit_b : (int)std::max(1LL, (1024 + ntri - 1) / ntri);
  pl.ns2 = std::min(pl.ns2, pl.pc);
  // Y: as many P-splits as fit the chip's resident blocks in one round (MI355X: 256 compute units;
  // the 128 x 128 bf16 tile runs two blocks per unit); the float64 form takes about 1024 blocks
  const long long t3 = (long long)cdiv(pl.nbf, ym) * cdiv(pl.nact, yn);
  const long long auto3 = pl.split ? std::max(1LL, (pl.yv == 1 ? 512 : 256) / t3) : std::max(1LL, (1024 + t3 - 1) / t3);
  pl.ns3 = tu.nsplit_y > 0 ? tu.nsplit_y : (int)auto3;
  pl.ns3 = std::min(pl.ns3, pl.pc);
  return pl;
}

struct Bufs {
  double *alpha, *beta, *HC, *Hpp, *J, *K, *Y2e, *Y, *D, *Kpart, *partials, *E, *dbuf;
  float* beta32;
  double* Ct;           // fp64
  u16 *cth, *ctl;       // split: bf16 C_A^T (the compact pair in the split mode)
  u16 *ch16, *cl16;     // split mode: fp16 pair of C~ sC
  uint32_t* bnd;        // split mode: scale bounds (call-level words, then two per chunk)
  float* colb;          // split mode: per-orbital bounds (4 nact)
  double *XT, *W, *Ypart64, *Bw;   // fp64 chunk
  float *Ct32, *XT32, *W32;        // fp32 path
  u16 *xth, *xtl, *wh, *wl, *bh, *bl;  // split chunk
  u16 *xth2, *xtl2;                    // split: XT of the next chunk (X runs one chunk ahead)
  float* Ypart32;
  double *Jr, *Kr;      // explicit integrals
  int* flag;
  size_t bytes;
};

Bufs carve(const Plan& pl, char* base) {
  Arena a(base);
  Bufs b{};
  const long long n2 = (long long)pl.nact * pl.nact;
  const long long ny = (long long)pl.nbf * pl.nact;
  b.alpha = a.take<double>(n2);
  b.beta = a.take<double>(n2);
  b.beta32 = a.take<float>(n2);
  b.HC = a.take<double>(ny);
  b.Hpp = a.take<double>(pl.nact);
  b.J = a.take<double>(n2);
  b.K = a.take<double>(n2);
  b.Y2e = a.take<double>(ny);
  b.Y = a.take<double>(ny);
  b.partials = a.take<double>(512);
  b.E = a.take<double>(4);
  b.flag = a.take<int>(4);
  if (is_df(pl.ints)) {
    b.D = a.take<double>((long long)pl.naux * pl.nact);
    b.dbuf = a.take<double>((long long)pl.pc * pl.nact);
    b.Kpart = a.take<double>((long long)pl.ns2 * n2);
    if (pl.f32) {
      b.Ct32 = a.take<float>((long long)pl.nact * pl.ldk);
      b.XT32 = a.take<float>((long long)pl.pc * pl.nact * pl.ldx);
      b.W32 = a.take<float>((long long)pl.pc * pl.nact * pl.ldw);
      b.Ypart32 = a.take<float>((long long)pl.ns3 * ny);
    } else if (!pl.split) {
      b.Ct = a.take<double>((long long)pl.nact * pl.ldk);
      b.XT = a.take<double>((long long)pl.pc * pl.nact * pl.ldx);
      b.W = a.take<double>((long long)pl.pc * pl.nact * pl.ldw);
      b.Ypart64 = a.take<double>((long long)pl.ns3 * ny);
      if (pl.ints == PNOF_INTS_DF_BF16) b.Bw = a.take<double>((long long)pl.pc * pl.nbf * pl.nbf);
    } else {
      b.cth = a.take<u16>((long long)pl.nact32 * pl.ldk);
      b.ctl = a.take<u16>((long long)pl.nact32 * pl.ldk);
      if (pl.terms > 1) {
        b.ch16 = a.take<u16>((long long)pl.nact32 * pl.ldk);
        b.cl16 = a.take<u16>((long long)pl.nact32 * pl.ldk);
        b.bnd = a.take<uint32_t>(scl_words(cdiv(pl.naux, pl.pc)));
        b.colb = a.take<float>(4LL * pl.nact);
      }
      b.xth = a.take<u16>((long long)pl.pc * pl.nact32 * pl.ldx);
      b.xth2 = a.take<u16>((long long)pl.pc * pl.nact32 * pl.ldx);
      b.wh = a.take<u16>((long long)pl.pc * pl.nact32 * pl.ldw);
      if (pl.terms > 1) {
        b.xtl = a.take<u16>((long long)pl.pc * pl.nact32 * pl.ldx);
        b.xtl2 = a.take<u16>((long long)pl.pc * pl.nact32 * pl.ldx);
        b.wl = a.take<u16>((long long)pl.pc * pl.nact32 * pl.ldw);
      }
      b.Ypart32 = a.take<float>((long long)pl.ns3 * ny);
      if (pl.ints == PNOF_INTS_DF_F64) {
        b.bh = a.take<u16>((long long)pl.pc * pl.nbf * pl.nbf);
        b.bl = a.take<u16>((long long)pl.pc * pl.nbf * pl.nbf);
      }
    }
  } else {
    b.Jr = a.take<double>((long long)pl.nact * pl.nbf * pl.nbf);
    b.Kr = a.take<double>((long long)pl.nact * pl.nbf * pl.nbf);
  }
  b.bytes = a.off + 256;
  return b;
}

// Workspace: the caller's if large enough, else the context's own (grow-only).
pnof_status get_ws(pnof_ctx ctx, size_t bytes, char** out) {
  if (ctx->ext_ws && ctx->ext_bytes >= bytes) { *out = ctx->ext_ws; return PNOF_OK; }
  if (ctx->own_bytes < bytes) {
    if (ctx->own_ws) {
      hipStreamSynchronize(ctx->stream);
      hipFree(ctx->own_ws);
      ctx->own_ws = nullptr;
      ctx->own_bytes = 0;
    }
    if (hipMalloc(&ctx->own_ws, bytes) != hipSuccess) {
      hipGetLastError();
      return fail(ctx, PNOF_E_NOMEM, "workspace allocation of " + std::to_string(bytes) + " bytes failed");
    }
    ctx->own_bytes = bytes;
  }
  *out = ctx->own_ws;
  return PNOF_OK;
}

pnof_status check_ctx(pnof_ctx ctx) {
  if (!ctx) return fail(nullptr, PNOF_E_ARG, "context is NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fail(ctx, PNOF_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
  e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, PNOF_E_DEVICE, std::string("earlier device error: ") + hipGetErrorString(e));
  return PNOF_OK;
}

pnof_status check_finite(pnof_ctx ctx, Bufs& b, const void* p, long long n, int is_bf16, const char* what) {
  DEV_CHECK(ctx, hipMemsetAsync(b.flag, 0, sizeof(int), ctx->stream));
  DEV_CHECK(ctx, count_nonfinite(ctx->stream, p, n, is_bf16, b.flag));
  int h = 0;
  DEV_CHECK(ctx, hipMemcpyAsync(&h, b.flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  DEV_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  if (h) return fail(ctx, PNOF_E_NONFINITE, std::string("non-finite value in ") + what);
  return PNOF_OK;
}

// ------------------------------------------------------------------------ the step driver
struct Req {
  double *J = nullptr, *K = nullptr, *Y = nullptr, *E = nullptr, *lam = nullptr, *dEdC = nullptr,
         *dEdn = nullptr, *asym = nullptr, *Hpp = nullptr;
  double *Jq = nullptr, *Kq = nullptr, *Fq = nullptr;
  const int32_t* q_idx = nullptr;
  int nq = 0;
  bool need_y = false;   // Fock vectors (and everything built from them)
  bool need_e = false;
  // a workspace given by the call (the pchunk is lowered until the plan fits; nothing is allocated),
  // and every step on the context's stream
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool one_stream = false;
};

// Float64 product C = A B with the strided views of gemm_f64 (A(m,k) = A[m*sam + k*sak], ...; one
// stride of each operand is 1), on the context stream.
pnof_status dprod(pnof_ctx ctx, int M, int N, int K, const double* A, long long sam, long long sak, const double* B,
                  long long sbk, long long sbn, double* C, long long scm, long long scn) {
  DEV_CHECK(ctx, gemm_f64(ctx->stream, M, N, K, 1, 1.0, A, sam, sak, 0, B, sbk, sbn, 0, 0.0, C, scm, scn, 0));
  return PNOF_OK;
}

pnof_status run_step(pnof_ctx ctx, const pnof_problem* prob, const double* C, const double* n,
                     const double* H, const void* ints, Req& r) {
  Plan pl = make_plan(prob, ctx->tune);
  Bufs b = carve(pl, nullptr);
  char* ws = nullptr;
  pnof_status st = PNOF_OK;
  if (r.ws) {
    // fit the caller's region: fewer rows of B per chunk until the plan's workspace fits
    pnof_tuning tu = ctx->tune;
    while (b.bytes > r.ws_bytes && pl.pc > 1) {
      tu.pchunk = std::max(1, pl.pc / 2);
      pl = make_plan(prob, tu);
      b = carve(pl, nullptr);
    }
    if (b.bytes > r.ws_bytes)
      return fail(ctx, PNOF_E_UNSUPPORTED,
                  "the problem needs " + std::to_string(b.bytes) + " bytes of workspace, more than the " +
                      std::to_string(r.ws_bytes) + " available");
    ws = r.ws;
  } else if ((st = get_ws(ctx, b.bytes, &ws)) != PNOF_OK) {
    return st;
  }
  b = carve(pl, ws);
  hipStream_t s = ctx->stream;
  const int nbf = pl.nbf, nact = pl.nact;
  const long long n2 = (long long)nact * nact, ny = (long long)nbf * nact;

  if (prob->flags & PNOF_CHECK_FINITE) {
    const long long nint = is_df(pl.ints) ? (long long)pl.naux * nbf * nbf : (long long)nbf * nbf * nbf * nbf;
    if ((st = check_finite(ctx, b, C, (long long)nbf * nbf, 0, "C")) != PNOF_OK) return st;
    if (n && (st = check_finite(ctx, b, n, nact, 0, "n")) != PNOF_OK) return st;
    if (H && (st = check_finite(ctx, b, H, (long long)nbf * nbf, 0, "H")) != PNOF_OK) return st;
    if ((st = check_finite(ctx, b, ints, nint, pl.ints == PNOF_INTS_DF_BF16, "integrals")) != PNOF_OK) return st;
  }

  double* J = r.J ? r.J : b.J;
  double* K = r.K ? r.K : b.K;
  double* Y = r.Y ? r.Y : b.Y;
  // the split and float32 modes correct the energy with Y (first order in the rounding of C)
  const bool want_y = r.need_y || ((pl.split || pl.f32) && r.need_e) || r.Fq;
  const bool want_e = r.need_e;
  const bool have_n = (n != nullptr);
  const OccLayout occ{n, pl.npairs, pl.ncwo, pl.nsingle};

  if (have_n) DEV_CHECK(ctx, coeffs(s, nact, pl.npairs, pl.ncwo, pl.nsingle, pl.functional, n, b.alpha, b.beta, b.beta32));
  if (H) {
    // HC = H C_A ; Hpp = diag(C_A^T H C_A)
    RB_CHECK(dprod(ctx, nbf, nact, nbf, H, nbf, 1, C, nbf, 1, b.HC, nact, 1));
    DEV_CHECK(ctx, hpp_from_hc(s, nbf, nact, C, b.HC, b.Hpp));
    if (r.Hpp) DEV_CHECK(ctx, hipMemcpyAsync(r.Hpp, b.Hpp, sizeof(double) * nact, hipMemcpyDeviceToDevice, s));
  }
  if (r.Jq) DEV_CHECK(ctx, fill_f64(s, r.Jq, (long long)r.nq * nbf * nbf, 0.0));
  if (r.Kq) DEV_CHECK(ctx, fill_f64(s, r.Kq, (long long)r.nq * nbf * nbf, 0.0));
  if (r.Fq) DEV_CHECK(ctx, fill_f64(s, r.Fq, (long long)r.nq * nbf * nbf, 0.0));

  int corr_terms = 0;
  if (!is_df(pl.ints)) {
    const double* ERI = static_cast<const double*>(ints);
    DEV_CHECK(ctx, eri_jk_ao(s, nbf, nact, ERI, C, b.Jr, b.Kr));
    DEV_CHECK(ctx, eri_jk_no(s, nbf, nact, C, b.Jr, b.Kr, J, K));
    if (want_y) DEV_CHECK(ctx, eri_y(s, nbf, nact, C, n, b.HC, b.alpha, b.beta, b.Jr, b.Kr, b.Y2e));
    if (r.Jq) DEV_CHECK(ctx, gather_ao(s, nbf, r.nq, r.q_idx, b.Jr, r.Jq));
    if (r.Kq) DEV_CHECK(ctx, gather_ao(s, nbf, r.nq, r.q_idx, b.Kr, r.Kq));
    if (r.Fq) DEV_CHECK(ctx, eri_fock_ao(s, nbf, nact, r.nq, r.q_idx, n, H, b.alpha, b.beta, b.Jr, b.Kr, r.Fq));
  } else {
    DEV_CHECK(ctx, fill_f64(s, K, n2, 0.0));
    DEV_CHECK(ctx, fill_f64(s, b.Kpart, (long long)pl.ns2 * n2, 0.0));
    if (want_y) DEV_CHECK(ctx, fill_f64(s, b.Y2e, ny, 0.0));
    WsDims wd{pl.nact32, 0, 0, 0};
    if (pl.f32) {
      DEV_CHECK(ctx, transpose_ca_f32(s, nbf, nact, C, b.Ct32, pl.ldk));
      corr_terms = 1;
    } else if (!pl.split) DEV_CHECK(ctx, transpose_ca(s, nbf, nact, C, b.Ct, pl.ldk));
    else {
      const long long nct = (long long)pl.nact32 * pl.ldk, nxt = (long long)pl.pc * pl.nact32 * pl.ldx,
                      nw = (long long)pl.pc * pl.nact32 * pl.ldw;
      wd = WsDims{pl.nact32, 2 * nct, 2 * nxt, 2 * nw};
      // the zero pads of the tiles are part of the contract of the contraction kernels; the valid
      // blocks (Ct: nact x nbf, XT_P: nact x nbf, W_P: the part of nact x nact that Y reads) are
      // overwritten before they are read, so only the pads are cleared
      const long long sx = (long long)pl.nact32 * pl.ldx, sw = (long long)pl.nact32 * pl.ldw;
      for (int lo = 0; lo < (pl.terms > 1 ? 2 : 1); ++lo) {
        DEV_CHECK(ctx, zero_pads_u16(s, lo ? b.ctl : b.cth, 1, nct, nact, pl.nact32, pl.ldk, nbf));
        if (pl.terms > 1) DEV_CHECK(ctx, zero_pads_u16(s, lo ? b.cl16 : b.ch16, 1, nct, nact, pl.nact32, pl.ldk, nbf));
        DEV_CHECK(ctx, zero_pads_u16(s, lo ? b.xtl : b.xth, pl.pc, sx, nact, pl.nact32, pl.ldx, nbf));
        DEV_CHECK(ctx, zero_pads_u16(s, lo ? b.xtl2 : b.xth2, pl.pc, sx, nact, pl.nact32, pl.ldx, nbf));
        DEV_CHECK(ctx, zero_pads_u16(s, lo ? b.wl : b.wh, pl.pc, sw, nact, pl.nact32, pl.ldw, nact));
      }
      // split mode: bounds that fix the power-of-two scales of the fp16 pairs (call-level words; the
      // per-chunk words are cleared here and raised by the row bounds of each chunk of B)
      if (pl.terms > 1)
        DEV_CHECK(ctx, scale_bounds(s, nbf, nact, C, n, pl.npairs, pl.ncwo, pl.nsingle, pl.functional, b.colb, b.bnd,
                                    2 * (int)cdiv(pl.naux, pl.pc)));
      DEV_CHECK(ctx, split_ca(s, nbf, nact, pl.terms, C, b.cth, b.ctl, b.ch16, b.cl16, pl.ldk, b.bnd));
      corr_terms = pl.terms > 1 ? 2 : 1;
    }
    const long long bsz = (long long)nbf * nbf;
    if (pl.f32) {
      for (int p0 = 0; p0 < pl.naux; p0 += pl.pc) {
        const int np = std::min(pl.pc, pl.naux - p0);
        const int ns2 = std::min(pl.ns2, np), ns3 = std::min(pl.ns3, np);
        double* Dc = b.D + (long long)p0 * nact;
        const bool bb = pl.ints == PNOF_INTS_DF_BF16;
        const void* Bc = bb ? static_cast<const void*>(static_cast<const u16*>(ints) + p0 * bsz)
                            : static_cast<const void*>(static_cast<const double*>(ints) + p0 * bsz);
        DEV_CHECK(ctx, TIMED(ctx, PNOF_STAGE_X, df_f32_gemm1(s, nbf, nact, np, b.Ct32, pl.ldk, Bc, bb, b.XT32, pl.ldx)));
        DEV_CHECK(ctx, TIMED(ctx, PNOF_STAGE_B, df_f32_gemm2(s, nbf, nact, np, ns2, b.Ct32, pl.ldk, b.XT32, pl.ldx,
                                                              b.beta32, b.Kpart, Dc, b.W32, pl.ldw)));
        if (want_y) {
          DEV_CHECK(ctx, add_diag_f32(s, nact, np, Dc, occ, b.dbuf, b.W32, pl.ldw));
          DEV_CHECK(ctx, TIMED(ctx, PNOF_STAGE_Y, df_f32_gemm3(s, nbf, nact, np, ns3, b.XT32, pl.ldx, b.W32, pl.ldw,
                                                                b.Ypart32)));
          DEV_CHECK(ctx, reduce_y_f32(s, ny, ns3, b.Ypart32, b.Y2e));
        }
        if (r.Jq || r.Kq || r.Fq)
          DEV_CHECK(ctx, df_ao_accum(s, nbf, nact, np, r.nq, r.q_idx, Bc, bb, Dc, b.alpha, b.beta, nullptr, b.XT32,
                                     nullptr, nullptr, pl.ldx, (long long)nact * pl.ldx, r.Jq, r.Kq, r.Fq, nullptr, 0));
      }
    } else if (!pl.split) {
      for (int p0 = 0; p0 < pl.naux; p0 += pl.pc) {
        const int np = std::min(pl.pc, pl.naux - p0);
        const int ns2 = std::min(pl.ns2, np), ns3 = std::min(pl.ns3, np);
        double* Dc = b.D + (long long)p0 * nact;
        const double* Bc;
        if (pl.ints == PNOF_INTS_DF_F64) Bc = static_cast<const double*>(ints) + p0 * bsz;
        else {
          DEV_CHECK(ctx, widen_bf16(s, np * bsz, static_cast<const u16*>(ints) + p0 * bsz, b.Bw));
          Bc = b.Bw;
        }
        DEV_CHECK(ctx, TIMED(ctx, PNOF_STAGE_X, df_f64_gemm1(s, nbf, nact, np, b.Ct, pl.ldk, Bc, b.XT, pl.ldx)));
        DEV_CHECK(ctx, TIMED(ctx, PNOF_STAGE_B, df_f64_gemm2(s, nbf, nact, np, ns2, b.Ct, pl.ldk, b.XT, pl.ldx, b.beta, b.Kpart, Dc, b.W, pl.ldw)));
        if (want_y) {
          DEV_CHECK(ctx, add_diag_f64(s, nact, np, Dc, occ, b.dbuf, b.W, pl.ldw));
          DEV_CHECK(ctx, TIMED(ctx, PNOF_STAGE_Y, df_f64_gemm3(s, nbf, nact, np, ns3, b.XT, pl.ldx, b.W, pl.ldw, b.Ypart64)));
          DEV_CHECK(ctx, reduce_y_f64(s, ny, ns3, b.Ypart64, b.Y2e));
        }
        if (r.Jq || r.Kq || r.Fq)
          DEV_CHECK(ctx, df_ao_accum(s, nbf, nact, np, r.nq, r.q_idx, Bc, 0, Dc, b.alpha, b.beta, b.XT, nullptr, nullptr,
                                     nullptr, pl.ldx, (long long)nact * pl.ldx, r.Jq, r.Kq, r.Fq, nullptr, 0));
      }
    } else {
      // Chunk pipeline: X of chunk c + 1 runs between b and Y of chunk c (XT is double-buffered,
      // chunk c in buffer c & 1), while the context's second stream forms chunk c's D alpha and W
      // diagonal beside X(c + 1), and reduces the Y partials of chunk c beside b and X of the next
      // chunks.  Events order the two streams: W's diagonal before Y(c); the reduction of Y(c - 1)
      // before Y(c) overwrites the partials; the last reduction before Y2e is read.  W itself is
      // single-buffered: Y(c) precedes b(c + 1) on the main stream.  Whatever path leaves this scope,
      // the main stream waits for the second one.
      const int nchunk = (int)cdiv(pl.naux, pl.pc);
      const bool split = pl.terms > 1;
      SplitPtr Ct{b.cth, split ? b.ctl : nullptr};      // X from a bf16 B: compact bf16 pair
      SplitPtr C16{split ? b.ch16 : b.cth, split ? b.cl16 : nullptr};   // b (and X from float64 B)
      u16* const xth_[2] = {b.xth, b.xth2};
      u16* const xtl_[2] = {b.xtl, b.xtl2};
      // W stored once per 128 x 128 block pair (b writes only the transposed image of its tiles, the
      // blocks on and above the diagonal; Y reads each block in the orientation that holds it): needs
      // Y's direct-load path
      auto a16 = [](const void* p) { return p == nullptr || (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
      const bool wsym = pl.ldx % 32 == 0 && pl.ldw % 32 == 0 && a16(b.xth) && a16(b.xth2) && a16(b.xtl) &&
                        a16(b.xtl2) && a16(b.wh) && a16(b.wl);
      // one_stream: the second stream's work runs in order on the context's stream
      const bool two = !r.one_stream;
      if (two) RB_CHECK(ensure_aux(ctx));
      AuxJoin join(ctx);
      hipStream_t sa = two ? ctx->aux : s;
      hipEvent_t ev_b = ctx->pipe_ev[0], ev_d = ctx->pipe_ev[1], ev_y = ctx->pipe_ev[2], ev_r = ctx->pipe_ev[3];
      auto chunk_rows = [&](int c) { return (int)std::min<long long>(pl.pc, pl.naux - (long long)c * pl.pc); };
      // row bounds of every chunk of B in one pass before the first X (beside the contractions it
      // would take their compute units: measured slower)
      if (split) {
        const auto& bd = ctx->bound;
        if (bd.ints && bd.ints == ints && bd.nbf == nbf && bd.naux == pl.naux && bd.kind == pl.ints && bd.pc == pl.pc)
          DEV_CHECK(ctx, hipMemcpyAsync(b.bnd + SCL_CALL, bd.words, bd.nwords * sizeof(uint32_t),
                                        hipMemcpyDeviceToDevice, s));   // bound integrals: kept bounds
        else
          DEV_CHECK(ctx, b_bounds(s, ints, pl.ints == PNOF_INTS_DF_F64, (long long)pl.naux * nbf, nbf, nbf,
                                  (long long)pl.pc * nbf, b.bnd + SCL_CALL));
      }
      auto run_x = [&](int c) -> pnof_status {
        const long long p0 = (long long)c * pl.pc;
        const int np = chunk_rows(c);
        SplitPtr Bp;
        SplitPtr A = Ct;
        long long b_bytes;
        if (pl.ints == PNOF_INTS_DF_BF16) {
          Bp.hi = static_cast<const u16*>(ints) + p0 * bsz;
          Bp.lo = nullptr;
          b_bytes = 2LL * (pl.naux - p0) * bsz;
        } else {
          b_bytes = 2LL * np * bsz;
          DEV_CHECK(ctx, split_b(s, np * bsz, static_cast<const double*>(ints) + p0 * bsz, b.bh, b.bl,
                                 split ? b.bnd : nullptr, c));
          Bp.hi = b.bh;
          Bp.lo = split ? b.bl : nullptr;
          if (split) A = C16;
        }
        DEV_CHECK(ctx, TIMED(ctx, PNOF_STAGE_X, df_bf16_gemm1(s, nbf, nact, np, pl.terms, A, pl.ldk, Bp, bsz, nbf, b_bytes,
                                                               xth_[c & 1], xtl_[c & 1], pl.ldx, pl.xv, wd, b.bnd, c)));
        return PNOF_OK;
      };
      RB_CHECK(run_x(0));
      for (int c = 0; c < nchunk; ++c) {
        const int p0 = c * pl.pc;
        const int np = chunk_rows(c);
        const int ns2 = std::min(pl.ns2, np), ns3 = std::min(pl.ns3, np);
        double* Dc = b.D + (long long)p0 * nact;
        SplitPtr XT{xth_[c & 1], split ? xtl_[c & 1] : nullptr};
        DEV_CHECK(ctx, TIMED(ctx, PNOF_STAGE_B, df_bf16_gemm2(s, nbf, nact, np, ns2, pl.terms, C16, pl.ldk, XT, pl.ldx,
                                                               b.beta32, b.Kpart, Dc, b.wh, b.wl, pl.ldw, wd, b.bnd, c,
                                                               wsym)));
        if (want_y) {
          if (two) {
            DEV_CHECK(ctx, hipEventRecord(ev_b, s));
            DEV_CHECK(ctx, hipStreamWaitEvent(sa, ev_b, 0));
            join.forked = true;
          }
          DEV_CHECK(ctx, add_diag_bf16(sa, nact, np, Dc, occ, b.beta32, b.dbuf, b.wh, b.wl, pl.ldw,
                                       (long long)pl.nact32 * pl.ldw, b.bnd, c));
          if (two) DEV_CHECK(ctx, hipEventRecord(ev_d, sa));
        }
        if (c + 1 < nchunk) RB_CHECK(run_x(c + 1));
        if (want_y) {
          if (two) {
            DEV_CHECK(ctx, hipStreamWaitEvent(s, ev_d, 0));
            if (c > 0) DEV_CHECK(ctx, hipStreamWaitEvent(s, ev_r, 0));
          }
          SplitPtr W{b.wh, b.wl};
          DEV_CHECK(ctx, TIMED(ctx, PNOF_STAGE_Y, df_bf16_gemm3(s, nbf, nact, np, ns3, pl.terms, XT, pl.ldx, W, pl.ldw,
                                                                 b.Ypart32, pl.yv, wd, b.bnd, c, wsym)));
          if (two) {
            DEV_CHECK(ctx, hipEventRecord(ev_y, s));
            DEV_CHECK(ctx, hipStreamWaitEvent(sa, ev_y, 0));
          }
          DEV_CHECK(ctx, reduce_y_f32(sa, ny, ns3, b.Ypart32, b.Y2e));
          if (two) DEV_CHECK(ctx, hipEventRecord(ev_r, sa));
        }
        if (r.Jq || r.Kq || r.Fq) {
          const void* Bsrc = pl.ints == PNOF_INTS_DF_BF16
                                 ? static_cast<const void*>(static_cast<const u16*>(ints) + (long long)p0 * bsz)
                                 : static_cast<const void*>(static_cast<const double*>(ints) + (long long)p0 * bsz);
          DEV_CHECK(ctx, df_ao_accum(s, nbf, nact, np, r.nq, r.q_idx, Bsrc, pl.ints == PNOF_INTS_DF_BF16, Dc, b.alpha,
                                     b.beta, nullptr, nullptr, XT.hi, XT.lo, pl.ldx, (long long)pl.nact32 * pl.ldx, r.Jq,
                                     r.Kq, r.Fq, b.bnd, c));
        }
      }
      if (want_y && two) DEV_CHECK(ctx, hipStreamWaitEvent(s, ev_r, 0));
    }
    DEV_CHECK(ctx, reduce_k(s, nact, pl.ns2, b.Kpart, K));
    // J = D^T D
    DEV_CHECK(ctx, gemm_f64(s, nact, nact, pl.naux, 1, 1.0, b.D, 1, nact, 0, b.D, nact, 1, 0, 0.0, J, nact, 1, 0));
    if (r.Fq) DEV_CHECK(ctx, fock_ao_h(s, nbf, r.nq, r.q_idx, n, H, r.Fq));
  }

  if (want_e) {
    double* E = r.E ? r.E : b.E;
    DEV_CHECK(ctx, energy(s, nbf, nact, n, b.Hpp, b.alpha, b.beta, J, K, b.Y2e, C, b.cth, b.ctl, b.Ct32, pl.ldk,
                          corr_terms, b.partials, E));
  }
  if (want_y) DEV_CHECK(ctx, assemble_y(s, nbf, nact, n, b.HC, b.Y2e, Y));
  if (r.lam) {
    RB_CHECK(dprod(ctx, nbf, nact, nbf, C, 1, nbf, Y, nact, 1, r.lam, nbf, 1));
    DEV_CHECK(ctx, zero_cols(s, nbf, nact, r.lam));
    if (r.asym) DEV_CHECK(ctx, max_asym(s, nbf, r.lam, b.partials + 256, r.asym));
  }
  if (r.dEdC) DEV_CHECK(ctx, grad_c(s, nbf, nact, Y, r.dEdC));
  if (r.dEdn) DEV_CHECK(ctx, grad_n(s, nact, pl.npairs, pl.ncwo, pl.nsingle, pl.functional, n, b.Hpp, J, K, r.dEdn));
  return PNOF_OK;
}

pnof_status check_ptrs(pnof_ctx ctx, std::initializer_list<const void*> ps, const char* what) {
  for (const void* p : ps)
    if (!p) return fail(ctx, PNOF_E_ARG, std::string("required pointer is NULL in ") + what);
  return PNOF_OK;
}

pnof_status check_q(pnof_ctx ctx, const void* a, const int32_t* q_idx, int32_t nq) {
  if (a && (!q_idx || nq <= 0)) return fail(ctx, PNOF_E_ARG, "per-orbital AO output needs q_idx and nq > 0");
  if (!a && nq < 0) return fail(ctx, PNOF_E_ARG, "nq must not be negative");
  return PNOF_OK;
}

}  // namespace

// ------------------------------------------------------------------------ batches
namespace {

// ------------------------------------------------------------------------ optimisation drivers
// Device buffers of one driver call, taken from the context's driver slots in call order (nested
// calls take the slots above their caller's); a slot is reallocated only when a call needs more than
// it holds (after the stream has drained), otherwise reused as is.
struct DevBuf {
  pnof_ctx ctx;
  size_t base;
  bool ok = true;
  explicit DevBuf(pnof_ctx c) : ctx(c), base(c->slot_top) {}
  ~DevBuf() { ctx->slot_top = base; }
  template <typename T>
  T* get(long long n) {
    const size_t bytes = sizeof(T) * (size_t)std::max(1LL, n);
    const size_t i = ctx->slot_top++;
    if (i == ctx->slots.size()) ctx->slots.push_back({nullptr, 0});
    pnof_ctx_s::Slot& sl = ctx->slots[i];
    if (sl.bytes < bytes) {
      if (sl.p) {
        hipStreamSynchronize(ctx->stream);
        hipFree(sl.p);
        sl.p = nullptr;
        sl.bytes = 0;
      }
      if (hipMalloc(&sl.p, bytes) != hipSuccess) {
        hipGetLastError();
        ok = false;
        return nullptr;
      }
      sl.bytes = bytes;
    }
    return static_cast<T*>(sl.p);
  }
};

// E(n(gamma)) and dE/dgamma at fixed H_pp, J, K, evaluated on the device (Section 3.1).
struct OnObjective {
  pnof_ctx ctx;
  int kind, npairs, ncwo, nsingle, nact, nbf, functional, ngam;
  const double *Hpp, *J, *K;
  double *gam, *n, *alpha, *beta, *partials, *E, *dEdn, *g;
  std::vector<double> host;
  int evals = 0;

  pnof_status eval(const std::vector<double>& x, double& f, std::vector<double>& grad) {
    hipStream_t s = ctx->stream;
    DEV_CHECK(ctx, hipMemcpyAsync(gam, x.data(), sizeof(double) * ngam, hipMemcpyHostToDevice, s));
    DEV_CHECK(ctx, on_map(s, kind, npairs, ncwo, nsingle, gam, n, nullptr));
    DEV_CHECK(ctx, coeffs(s, nact, npairs, ncwo, nsingle, functional, n, alpha, beta, nullptr));
    DEV_CHECK(ctx, energy(s, nbf, nact, n, Hpp, alpha, beta, J, K, nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0,
                          partials, E));
    DEV_CHECK(ctx, grad_n(s, nact, npairs, ncwo, nsingle, functional, n, Hpp, J, K, dEdn));
    DEV_CHECK(ctx, on_map_vjp(s, kind, npairs, ncwo, nsingle, gam, dEdn, g));
    host.resize(ngam + 1);
    DEV_CHECK(ctx, hipMemcpyAsync(host.data(), E, sizeof(double), hipMemcpyDeviceToHost, s));
    DEV_CHECK(ctx, hipMemcpyAsync(host.data() + 1, g, sizeof(double) * ngam, hipMemcpyDeviceToHost, s));
    DEV_CHECK(ctx, hipStreamSynchronize(s));
    f = host[0];
    grad.assign(host.begin() + 1, host.end());
    ++evals;
    if (!std::isfinite(f)) return fail(ctx, PNOF_E_NONFINITE, "occupation optimisation reached a non-finite energy");
    return PNOF_OK;
  }
};

pnof_status on_objective_init(pnof_ctx ctx, DevBuf& db, const pnof_problem* prob, int kind, const double* Hpp,
                              const double* J, const double* K, OnObjective& o) {
  o.ctx = ctx;
  o.kind = kind;
  o.npairs = prob->npairs;
  o.ncwo = prob->ncwo;
  o.nsingle = prob->nsingle;
  o.nact = prob->npairs * (prob->ncwo + 1) + prob->nsingle;
  o.nbf = prob->nbf;
  o.functional = prob->functional;
  o.ngam = kind == 0 ? o.nact : o.npairs * o.ncwo;
  o.Hpp = Hpp;
  o.J = J;
  o.K = K;
  const long long n2 = (long long)o.nact * o.nact;
  o.gam = db.get<double>(o.ngam);
  o.n = db.get<double>(o.nact);
  o.alpha = db.get<double>(n2);
  o.beta = db.get<double>(n2);
  o.partials = db.get<double>(512);
  o.E = db.get<double>(4);
  o.dEdn = db.get<double>(o.nact);
  o.g = db.get<double>(o.ngam);
  if (!db.ok) return fail(ctx, PNOF_E_NOMEM, "allocation of the occupation-optimisation buffers failed");
  return PNOF_OK;
}

double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

// Limited-memory BFGS (two-loop recursion) with a backtracking Armijo line search.
pnof_status lbfgs(OnObjective& o, std::vector<double>& x, const pnof_on_opts& op, double& fx, int& iters) {
  const int m = op.memory > 0 ? op.memory : 10;
  const int maxit = op.maxiter > 0 ? op.maxiter : 1000;
  const double gtol = op.gtol > 0 ? op.gtol : 1e-9;
  const size_t nv = x.size();
  std::vector<double> g, xn(nv), gn, d(nv);
  std::vector<std::vector<double>> S, Y;
  std::vector<double> rho;
  pnof_status st = o.eval(x, fx, g);
  if (st != PNOF_OK) return st;
  int it = 0, stalled = 0;
  for (; it < maxit; ++it) {
    double gmax = 0.0;
    for (double v : g) gmax = std::max(gmax, std::fabs(v));
    if (gmax <= gtol) break;
    // two-loop recursion: d = -H g
    std::vector<double> q = g, a(S.size());
    for (int i = (int)S.size() - 1; i >= 0; --i) {
      a[i] = rho[i] * dot(S[i], q);
      for (size_t k = 0; k < nv; ++k) q[k] -= a[i] * Y[i][k];
    }
    const double h0 = S.empty() ? 1.0 / std::max(1.0, gmax) : dot(S.back(), Y.back()) / dot(Y.back(), Y.back());
    for (size_t k = 0; k < nv; ++k) q[k] *= h0;
    for (size_t i = 0; i < S.size(); ++i) {
      const double bcoef = rho[i] * dot(Y[i], q);
      for (size_t k = 0; k < nv; ++k) q[k] += S[i][k] * (a[i] - bcoef);
    }
    for (size_t k = 0; k < nv; ++k) d[k] = -q[k];
    double gd = dot(g, d);
    if (!(gd < 0.0)) {   // not a descent direction: restart from the scaled gradient
      S.clear();
      Y.clear();
      rho.clear();
      for (size_t k = 0; k < nv; ++k) d[k] = -g[k] / std::max(1.0, gmax);
      gd = dot(g, d);
    }
    double step = 1.0, fn = fx;
    bool accepted = false;
    for (int ls = 0; ls < 60; ++ls) {
      for (size_t k = 0; k < nv; ++k) xn[k] = x[k] + step * d[k];
      if ((st = o.eval(xn, fn, gn)) != PNOF_OK) return st;
      if (fn <= fx + 1e-4 * step * gd) {
        accepted = true;
        break;
      }
      step *= 0.5;
    }
    if (!accepted) break;   // no decrease along d within rounding: the minimum is reached
    std::vector<double> sv(nv), yv(nv);
    for (size_t k = 0; k < nv; ++k) {
      sv[k] = xn[k] - x[k];
      yv[k] = gn[k] - g[k];
    }
    const double sy = dot(sv, yv);
    if (sy > 1e-14 * std::sqrt(dot(sv, sv) * dot(yv, yv))) {
      S.push_back(sv);
      Y.push_back(yv);
      rho.push_back(1.0 / sy);
      if ((int)S.size() > m) {
        S.erase(S.begin());
        Y.erase(Y.begin());
        rho.erase(rho.begin());
      }
    }
    // stagnation: three successive steps that change E by no more than its rounding
    stalled = (fx - fn <= 4.0 * DBL_EPSILON * std::max(1.0, std::fabs(fx))) ? stalled + 1 : 0;
    x = xn;
    g = gn;
    fx = fn;
    if (stalled >= 3) break;
  }
  iters = it;
  return PNOF_OK;
}

// H_pp = diag(C_A^T H C_A) into Hpp (device), through the scratch HC (nbf x nact).
pnof_status hpp_of(pnof_ctx ctx, int nbf, int nact, const double* C, const double* H, double* HC, double* Hpp) {
  hipStream_t s = ctx->stream;
  DEV_CHECK(ctx, gemm_f64(s, nbf, nact, nbf, 1, 1.0, H, nbf, 1, 0, C, nbf, 1, 0, 0.0, HC, nact, 1, 0));
  DEV_CHECK(ctx, hpp_from_hc(s, nbf, nact, C, HC, Hpp));
  return PNOF_OK;
}

// Small dense solve (Gaussian elimination with partial pivoting), row-major A (n x n).
bool solve_small(std::vector<double> A, std::vector<double>& b, int n) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (std::fabs(A[piv * n + c]) < 1e-300) return false;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      const double f = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      b[r] -= f * b[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double v = b[r];
    for (int k = r + 1; k < n; ++k) v -= A[r * n + k] * b[k];
    b[r] = v / A[r * n + r];
  }
  return true;
}

// Geometry of one batch instance: sizes, leading dimensions and P-splits of the grouped launches.
struct BatchGeom {
  int nbf, nact, naux, ldk, ldw, nact32, ns2, ns3;
};

BatchGeom batch_geom(const pnof_problem& p) {
  BatchGeom g{};
  g.nbf = p.nbf;
  g.nact = p.npairs * (p.ncwo + 1) + p.nsingle;
  g.naux = p.naux;
  g.ldk = (int)round_up(g.nbf, 32);
  g.nact32 = g.ldw = (int)round_up(g.nact, 32);
  // P-splits sized so that one work item of the b and Y contractions is about 64 k-tiles long
  const int pps2 = std::max(1, 64 / cdiv(g.nbf, 32)), pps3 = std::max(1, 64 / cdiv(g.nact, 32));
  g.ns2 = cdiv(g.naux, pps2);
  g.ns3 = cdiv(g.naux, pps3);
  return g;
}

}  // namespace

struct pnof_batch_s {
  pnof_ctx ctx = nullptr;
  int ninst = 0, terms = 3;
  std::vector<pnof_problem> probs;
  std::vector<BatchGeom> geo;
  std::vector<BInst> inst;            // host copies (pointers filled at plan and bind)
  char* ws = nullptr;
  size_t bytes = 0;
  BInst* d_inst = nullptr;
  G1Args* d_g1 = nullptr;
  G2Args* d_g2 = nullptr;
  G3Args* d_g3 = nullptr;
  int* d_off = nullptr;               // 3 x (ninst + 1)
  F64Gemm* d_f64 = nullptr;           // 4 x ninst: H C_A, D alpha, D^T D, C^T Y
  int tot1 = 0, tot2 = 0, tot3 = 0;
  BMax mx{};
  int maxM[4] = {0, 0, 0, 0}, maxN[4] = {0, 0, 0, 0};
  bool bound = false;
  hipStream_t cap = nullptr;
  hipStream_t side = nullptr;         // second stream of a step (default priority)
  hipEvent_t ev[3] = {};              // fork at the start, fork after b, join before energy_y
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int launches = 13;
  int req[3] = {0, 0, 0};             // requested tile widths along the active orbitals (0: automatic)
  int tile[3] = {128, 128, 128};      // in use: X (rows p), b (square), Y (columns q)
  // persistent kernel: scheduling state (batch workspace), its graph, the last run's mode
  PSched ps{};
  int* d_cnt = nullptr;
  int* d_order = nullptr;             // instances grouped by die (see batch_offsets)
  int* d_xoff = nullptr;
  hipGraph_t pgraph = nullptr;
  hipGraphExec_t pexec = nullptr;
  int pblocks = 512;                  // two blocks per compute unit
  double stall_us = 1e6;              // no progress for this long: a persistent run gives up
  int dev_dies = 1;                   // the device's XCC count
  int last_flags = -1;
  double clock_khz = 0.0;             // device wall clock
};

namespace {

void batch_drop_graph(pnof_batch b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->pexec) hipGraphExecDestroy(b->pexec);
  if (b->pgraph) hipGraphDestroy(b->pgraph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->pexec = nullptr;
  b->pgraph = nullptr;
}

// The fixed launch sequence of one batch step.
// Tile widths along the active orbitals for the grouped X, b and Y contractions.  Automatic: 64
// when it cuts the padded matrix-core work of that stage, summed over the instances, by a quarter or
// more (the 64-wide forms do less work per LDS byte, so a small saving does not pay).
void batch_resolve_tiles(pnof_batch b) {
  double w[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  const int ts[2] = {128, 64};
  for (const BatchGeom& g : b->geo)
    for (int k = 0; k < 2; ++k) {
      const double t = ts[k], na = (double)round_up(g.nact, ts[k]), tt = cdiv(g.nact, ts[k]);
      w[0][k] += (double)g.naux * g.nbf * g.ldk * na;
      w[1][k] += (double)g.naux * g.ldk * t * t * tt * (tt + 1) / 2;
      w[2][k] += (double)g.naux * round_up(g.nbf, 128) * na * g.nact32;
    }
  for (int s = 0; s < 3; ++s) b->tile[s] = b->req[s] ? b->req[s] : (w[s][1] <= 0.75 * w[s][0] ? 64 : 128);
}

// Work-item offsets of the grouped launches for the tiles in use (the kernels decode with the same
// widths), uploaded to the device.
hipError_t batch_offsets(pnof_batch b, hipStream_t s) {
  const int n = b->ninst;
  std::vector<int> off(3 * (n + 1), 0);
  for (int i = 0; i < n; ++i) {
    const BatchGeom& g = b->geo[i];
    G1Args g1{};
    g1.nbf = g.nbf; g1.nact = g.nact; g1.np = g.naux;
    G2Args g2{};
    g2.nact = g.nact; g2.nsplit = g.ns2;
    G3Args g3{};
    g3.nbf = g.nbf; g3.nact = g.nact; g3.nsplit = g.ns3;
    off[i + 1] = off[i] + g1_items(g1, b->tile[0], 128, true);
    off[(n + 1) + i + 1] = off[(n + 1) + i] + g2_items(g2, b->tile[1]);
    off[2 * (n + 1) + i + 1] = off[2 * (n + 1) + i] + g3_items(g3, 128, b->tile[2]);
  }
  b->tot1 = off[n];
  b->tot2 = off[2 * (n + 1) - 1];
  b->tot3 = off[3 * (n + 1) - 1];
  // work items per phase of the persistent kernel (X and Y at the widths in use, b 64-wide)
  std::vector<int> cnt((size_t)n * PH_N);
  for (int i = 0; i < n; ++i) {
    const BatchGeom& g = b->geo[i];
    G1Args g1{};
    g1.nbf = g.nbf; g1.nact = g.nact; g1.np = g.naux;
    G2Args g2{};
    g2.nact = g.nact; g2.nsplit = g.ns2;
    G3Args g3{};
    g3.nbf = g.nbf; g3.nact = g.nact; g3.nsplit = g.ns3;
    persist_counts(b->inst[i], g1, g2, g3, b->tile[0], b->tile[2], cnt.data() + (size_t)i * PH_N);
  }
  // the persistent kernel runs each instance on one die: longest-first assignment of the instances'
  // contraction work to the least loaded die, each die's instances in index order
  std::vector<double> work(n);
  for (int i = 0; i < n; ++i) {
    const BatchGeom& g = b->geo[i];
    work[i] = 2.0 * g.naux * g.nbf * g.nact * (g.nbf + 2.0 * g.nact);
  }
  std::vector<int> byw(n);
  for (int i = 0; i < n; ++i) byw[i] = i;
  std::stable_sort(byw.begin(), byw.end(), [&](int x, int y) { return work[x] > work[y]; });
  const int nd = b->ps.ndie;
  std::vector<std::vector<int>> die(nd);
  std::vector<double> load(nd, 0.0);
  for (int i : byw) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    die[x].push_back(i);
    load[x] += work[i];
  }
  std::vector<int> order, xoff(nd + 1, 0);
  for (int x = 0; x < nd; ++x) {
    std::sort(die[x].begin(), die[x].end());
    order.insert(order.end(), die[x].begin(), die[x].end());
    xoff[x + 1] = (int)order.size();
  }
  hipError_t e = hipMemcpyAsync(b->d_off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(b->d_cnt, cnt.data(), sizeof(int) * cnt.size(), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(b->d_order, order.data(), sizeof(int) * n, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(b->d_xoff, xoff.data(), sizeof(int) * xoff.size(), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);   // off and cnt go out of scope
}

// Two branches, forked and joined with events (in a captured graph they become parallel nodes):
// H C_A and H_pp, which only the energy reads, run on the side stream beside prep, X and b; then
// J = D^T D beside D alpha, W's diagonal, Y and the reduction.
hipError_t batch_enqueue(pnof_batch b, hipStream_t s) {
  const int n = b->ninst;
  hipStream_t s2 = b->side;
  hipError_t e;
#define BSTEP(expr) \
  if ((e = (expr)) != hipSuccess) return e
  BSTEP(hipEventRecord(b->ev[0], s));
  BSTEP(hipStreamWaitEvent(s2, b->ev[0], 0));
  BSTEP(gemm_f64_grouped(s2, n, b->maxM[0], b->maxN[0], false, true, b->d_f64));
  BSTEP(batch_hpp(s2, n, b->d_inst, b->mx));
  if (b->terms > 1) BSTEP(batch_bounds(s, n, b->d_inst, b->mx));
  BSTEP(batch_prep(s, n, b->d_inst, b->mx));
  BSTEP(df_bf16_gemm1_grouped(s, n, b->tot1, b->terms, b->tile[0], b->d_g1, b->d_off));
  BSTEP(df_bf16_gemm2_grouped(s, n, b->tot2, b->terms, b->tile[1], b->d_g2, b->d_off + (n + 1)));
  BSTEP(hipEventRecord(b->ev[1], s));
  BSTEP(hipStreamWaitEvent(s2, b->ev[1], 0));
  BSTEP(gemm_f64_grouped(s2, n, b->maxM[2], b->maxN[2], true, true, b->d_f64 + 2 * n));
  BSTEP(hipEventRecord(b->ev[2], s2));
  BSTEP(gemm_f64_grouped(s, n, b->maxM[1], b->maxN[1], false, true, b->d_f64 + n));
  BSTEP(batch_add_diag(s, n, b->d_inst, b->mx));
  BSTEP(df_bf16_gemm3_grouped(s, n, b->tot3, b->terms, b->tile[2], b->d_g3, b->d_off + 2 * (n + 1)));
  BSTEP(batch_reduce(s, n, b->d_inst, b->mx));
  BSTEP(hipStreamWaitEvent(s, b->ev[2], 0));
  BSTEP(batch_energy_y(s, n, b->d_inst, b->mx));
  BSTEP(gemm_f64_grouped(s, n, b->maxM[3], b->maxN[3], true, true, b->d_f64 + 3 * n));
  BSTEP(batch_finish(s, n, b->d_inst, b->mx));
  BSTEP(batch_vjp(s, n, b->d_inst, b->mx));
#undef BSTEP
  return hipSuccess;
}

// The persistent form: one launch clears the scheduling state, one runs every step of every instance.
hipError_t batch_enqueue_persistent(pnof_batch b, hipStream_t s) {
  PArgs a{};
  a.ninst = b->ninst;
  a.terms = b->terms;
  a.inst = b->d_inst;
  a.g1 = b->d_g1;
  a.g2 = b->d_g2;
  a.g3 = b->d_g3;
  a.f64 = b->d_f64;
  a.sc = b->ps;
  a.sc.stall_ticks = (unsigned long long)(b->stall_us * b->clock_khz * 1e-3) + 1;
  return batch_persist(s, a, b->ninst * PH_N, b->tile[0], b->tile[2], b->pblocks);
}

pnof_status batch_fail(pnof_batch b, pnof_status st, const std::string& msg) { return fail(b ? b->ctx : nullptr, st, msg); }

}  // namespace

// ============================================================================ ABI
extern "C" {

int pnof_abi_version(void) { return PNOF_ABI_VERSION; }

const char* pnof_last_error(pnof_ctx ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

pnof_status pnof_check_problem(const pnof_problem* prob) { return check_problem(nullptr, prob); }

pnof_status pnof_create(pnof_ctx* out, int device, void* hip_stream) {
  if (!out) return fail(nullptr, PNOF_E_ARG, "output pointer is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    hipGetLastError();
    return fail(nullptr, PNOF_E_DEVICE, "no HIP device");
  }
  if (device < 0 || device >= ndev) return fail(nullptr, PNOF_E_ARG, "device index out of range");
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, PNOF_E_DEVICE, "hipSetDevice failed");
  pnof_ctx c = new pnof_ctx_s();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (rocblas_create_handle(&c->blas) != rocblas_status_success) {
    delete c;
    return fail(nullptr, PNOF_E_DEVICE, "rocblas_create_handle failed");
  }
  rocblas_set_stream(c->blas, c->stream);
  {
    // device address of the static workspace of pnof_lagrangian_noalloc on this device
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < kMaxDevices && !g_scratch[device]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        hipGetLastError();
        rocblas_destroy_handle(c->blas);
        delete c;
        return fail(nullptr, PNOF_E_DEVICE, std::string("hipGetSymbolAddress of the static workspace: ") +
                                                hipGetErrorString(e));
      }
      g_scratch[device] = p;
    }
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&c->host_info), sizeof(int) * 4, hipHostMallocDefault) != hipSuccess) {
    rocblas_destroy_handle(c->blas);
    delete c;
    return fail(nullptr, PNOF_E_NOMEM, "pinned allocation failed");
  }
  *out = c;
  return PNOF_OK;
}

void pnof_destroy(pnof_ctx ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  for (auto& e : ctx->evs) {
    hipEventDestroy(e.a);
    hipEventDestroy(e.b);
  }
  for (auto e : ctx->pool) hipEventDestroy(e);
  for (auto& sl : ctx->slots)
    if (sl.p) hipFree(sl.p);
  if (ctx->aux) {
    hipStreamSynchronize(ctx->aux);
    hipStreamDestroy(ctx->aux);
  }
  if (ctx->fork_ev) hipEventDestroy(ctx->fork_ev);
  if (ctx->join_ev) hipEventDestroy(ctx->join_ev);
  for (hipEvent_t e : ctx->pipe_ev)
    if (e) hipEventDestroy(e);
  if (ctx->own_ws) hipFree(ctx->own_ws);
  if (ctx->bound.words) hipFree(ctx->bound.words);
  if (ctx->host_info) hipHostFree(ctx->host_info);
  if (ctx->blas) rocblas_destroy_handle(ctx->blas);
  delete ctx;
}

pnof_status pnof_set_stream(pnof_ctx ctx, void* hip_stream) {
  if (!ctx) return fail(nullptr, PNOF_E_ARG, "context is NULL");
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  rocblas_set_stream(ctx->blas, ctx->stream);
  return PNOF_OK;
}

pnof_status pnof_workspace_size(pnof_ctx ctx, const pnof_problem* prob, size_t* bytes) {
  pnof_status st = check_problem(ctx, prob);
  if (st != PNOF_OK) return st;
  if (!bytes) return fail(ctx, PNOF_E_ARG, "bytes is NULL");
  *bytes = carve(make_plan(prob, ctx ? ctx->tune : pnof_tuning{0, 0, 0, 0, 0}), nullptr).bytes;
  return PNOF_OK;
}

pnof_status pnof_set_workspace(pnof_ctx ctx, void* dev, size_t bytes) {
  if (!ctx) return fail(nullptr, PNOF_E_ARG, "context is NULL");
  if (dev && (reinterpret_cast<uintptr_t>(dev) & 255)) return fail(ctx, PNOF_E_ARG, "workspace must be 256-byte aligned");
  ctx->ext_ws = static_cast<char*>(dev);
  ctx->ext_bytes = dev ? bytes : 0;
  return PNOF_OK;
}

pnof_status pnof_profile_begin(pnof_ctx ctx) {
  if (!ctx) return fail(nullptr, PNOF_E_ARG, "context is NULL");
  for (auto& e : ctx->evs) {
    ctx->pool.push_back(e.a);
    ctx->pool.push_back(e.b);
  }
  ctx->evs.clear();
  ctx->profiling = true;
  return PNOF_OK;
}

pnof_status pnof_profile_end(pnof_ctx ctx, double* ms, int64_t* launches) {
  if (!ctx) return fail(nullptr, PNOF_E_ARG, "context is NULL");
  if (!ms || !launches) return fail(ctx, PNOF_E_ARG, "output arrays are NULL");
  ctx->profiling = false;
  for (int i = 0; i < PNOF_NSTAGES; ++i) { ms[i] = 0.0; launches[i] = 0; }
  DEV_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& e : ctx->evs) {
    float t = 0.f;
    DEV_CHECK(ctx, hipEventElapsedTime(&t, e.a, e.b));
    ms[e.stage] += t;
    launches[e.stage] += 1;
    ctx->pool.push_back(e.a);
    ctx->pool.push_back(e.b);
  }
  ctx->evs.clear();
  return PNOF_OK;
}

pnof_status pnof_set_pchunk(pnof_ctx ctx, int32_t pchunk) {
  if (!ctx) return fail(nullptr, PNOF_E_ARG, "context is NULL");
  if (pchunk < 0) return fail(ctx, PNOF_E_ARG, "pchunk must be >= 0");
  ctx->tune.pchunk = pchunk;
  return PNOF_OK;
}

pnof_status pnof_set_tuning(pnof_ctx ctx, const pnof_tuning* t) {
  if (!ctx) return fail(nullptr, PNOF_E_ARG, "context is NULL");
  if (!t) {
    ctx->tune = pnof_tuning{0, 0, 0, 0, 0};
    return PNOF_OK;
  }
  if (t->pchunk < 0 || t->nsplit_b < 0 || t->nsplit_y < 0 || t->x_variant < 0 || t->x_variant > 3 ||
      t->y_variant < 0 || t->y_variant > 3)
    return fail(ctx, PNOF_E_ARG, "tuning values out of range");
  ctx->tune = *t;
  return PNOF_OK;
}

pnof_status pnof_bind_integrals(pnof_ctx ctx, const pnof_problem* prob, const void* ints) {
  if (!ctx) return fail(nullptr, PNOF_E_ARG, "context is NULL");
  auto& bd = ctx->bound;
  bd.ints = nullptr;
  if (!prob || !ints) return PNOF_OK;
  pnof_status st = check_problem(ctx, prob);
  if (st != PNOF_OK) return st;
  if ((st = check_ptrs(ctx, {ints}, "pnof_bind_integrals")) != PNOF_OK) return st;
  if ((st = check_ctx(ctx)) != PNOF_OK) return st;
  const Plan pl = make_plan(prob, ctx->tune);
  if (!is_df(pl.ints) || pl.terms <= 1) return PNOF_OK;
  const size_t nw = 2 * (size_t)cdiv(pl.naux, pl.pc);
  if (nw > bd.cap) {
    if (bd.words) DEV_CHECK(ctx, hipFree(bd.words));
    bd.words = nullptr;
    bd.cap = 0;
    DEV_CHECK(ctx, hipMalloc(&bd.words, nw * sizeof(uint32_t)));
    bd.cap = nw;
  }
  hipStream_t s = ctx->stream;
  DEV_CHECK(ctx, hipMemsetAsync(bd.words, 0, nw * sizeof(uint32_t), s));   // the bounds are raised from zero
  DEV_CHECK(ctx, b_bounds(s, ints, pl.ints == PNOF_INTS_DF_F64, (long long)pl.naux * pl.nbf, pl.nbf, pl.nbf,
                          (long long)pl.pc * pl.nbf, bd.words));
  bd.ints = ints;
  bd.nbf = pl.nbf;
  bd.naux = pl.naux;
  bd.kind = pl.ints;
  bd.pc = pl.pc;
  bd.nwords = nw;
  return PNOF_OK;
}

pnof_status pnof_get_plan(pnof_ctx ctx, const pnof_problem* prob, pnof_tuning* out) {
  if (!ctx) return fail(nullptr, PNOF_E_ARG, "context is NULL");
  pnof_status st = check_problem(ctx, prob);
  if (st != PNOF_OK) return st;
  if (!out) return fail(ctx, PNOF_E_ARG, "output is NULL");
  const Plan pl = make_plan(prob, ctx->tune);
  *out = pnof_tuning{pl.pc, pl.ns2, pl.ns3, pl.xv, pl.yv};
  return PNOF_OK;
}

pnof_status pnof_on_map(pnof_ctx ctx, int32_t kind, int32_t npairs, int32_t ncwo, int32_t nsingle,
                        const double* gamma, double* n, double* dn_dgamma) {
  if (!ctx) return fail(nullptr, PNOF_E_ARG, "context is NULL");
  if (kind != 0 && kind != 1) return fail(ctx, PNOF_E_ARG, "unknown ON map kind");
  if (npairs <= 0 || ncwo <= 0) return fail(ctx, PNOF_E_SHAPE, "npairs and ncwo must be positive");
  pnof_status st = check_ptrs(ctx, {gamma, n}, "pnof_on_map");
  if (st != PNOF_OK) return st;
  if ((st = check_ctx(ctx)) != PNOF_OK) return st;
  if (nsingle < 0) return fail(ctx, PNOF_E_SHAPE, "nsingle must not be negative");
  const long long nact = (long long)npairs * (ncwo + 1) + nsingle;
  const long long ngam = kind == 0 ? nact : (long long)npairs * ncwo;
  if (dn_dgamma) DEV_CHECK(ctx, fill_f64(ctx->stream, dn_dgamma, nact * ngam, 0.0));
  DEV_CHECK(ctx, on_map(ctx->stream, kind, npairs, ncwo, nsingle, gamma, n, dn_dgamma));
  return PNOF_OK;
}

pnof_status pnof_on_map_vjp(pnof_ctx ctx, int32_t kind, int32_t npairs, int32_t ncwo, int32_t nsingle,
                            const double* gamma, const double* dEdn, double* dEdgamma) {
  if (!ctx) return fail(nullptr, PNOF_E_ARG, "context is NULL");
  if (kind != 0 && kind != 1) return fail(ctx, PNOF_E_ARG, "unknown ON map kind");
  if (npairs <= 0 || ncwo <= 0) return fail(ctx, PNOF_E_SHAPE, "npairs and ncwo must be positive");
  pnof_status st = check_ptrs(ctx, {gamma, dEdn, dEdgamma}, "pnof_on_map_vjp");
  if (st != PNOF_OK) return st;
  if ((st = check_ctx(ctx)) != PNOF_OK) return st;
  if (nsingle < 0) return fail(ctx, PNOF_E_SHAPE, "nsingle must not be negative");
  DEV_CHECK(ctx, on_map_vjp(ctx->stream, kind, npairs, ncwo, nsingle, gamma, dEdn, dEdgamma));
  return PNOF_OK;
}

pnof_status pnof_jk(pnof_ctx ctx, const pnof_problem* prob, const double* C, const void* ints, double* J, double* K,
                    double* Jq_ao, double* Kq_ao, const int32_t* q_idx, int32_t nq) {
  if (!ctx) return fail(nullptr, PNOF_E_ARG, "context is NULL");
  pnof_status st = check_problem(ctx, prob);
  if (st != PNOF_OK) return st;
  if ((st = check_ptrs(ctx, {C, ints, J, K}, "pnof_jk")) != PNOF_OK) return st;
  if ((!Jq_ao) != (!Kq_ao)) return fail(ctx, PNOF_E_ARG, "Jq_ao and Kq_ao must both be set or both be NULL");
  if ((st = check_q(ctx, Jq_ao, q_idx, nq)) != PNOF_OK) return st;
  if ((st = check_ctx(ctx)) != PNOF_OK) return st;
  Req r;
  r.J = J;
  r.K = K;
  r.Jq = Jq_ao;
  r.Kq = Kq_ao;
  r.q_idx = q_idx;
  r.nq = Jq_ao ? nq : 0;
  // the coefficient kernels are not needed; pass no ONs
  return run_step(ctx, prob, C, nullptr, nullptr, ints, r);
}

pnof_status pnof_energy(pnof_ctx ctx, const pnof_problem* prob, const double* C, const double* n, const double* H,
                        const void* ints, double* E) {
  if (!ctx) return fail(nullptr, PNOF_E_ARG, "context is NULL");
  pnof_status st = check_problem(ctx, prob);
  if (st != PNOF_OK) return st;
  if ((st = check_ptrs(ctx, {C, n, H, ints, E}, "pnof_energy")) != PNOF_OK) return st;
  if ((st = check_ctx(ctx)) != PNOF_OK) return st;
  Req r;
  r.E = E;
  r.need_e = true;
  return run_step(ctx, prob, C, n, H, ints, r);
}

pnof_status pnof_fock(pnof_ctx ctx, const pnof_problem* prob, const double* C, const double* n, const double* H,
                      const void* ints, double* Y, double* Fq_ao, const int32_t* q_idx, int32_t nq) {
  if (!ctx) return fail(nullptr, PNOF_E_ARG, "context is NULL");
  pnof_status st = check_problem(ctx, prob);
  if (st != PNOF_OK) return st;
  if ((st = check_ptrs(ctx, {C, n, H, ints, Y}, "pnof_fock")) != PNOF_OK) return st;
  if ((st = check_q(ctx, Fq_ao, q_idx, nq)) != PNOF_OK) return st;
  if ((st = check_ctx(ctx)) != PNOF_OK) return st;
  Req r;
  r.Y = Y;
  r.need_y = true;
  r.Fq = Fq_ao;
  r.q_idx = q_idx;
  r.nq = Fq_ao ? nq : 0;
  return run_step(ctx, prob, C, n, H, ints, r);
}

pnof_status pnof_lagrangian(pnof_ctx ctx, const pnof_problem* prob, const double* C, const double* n,
                            const double* H, const void* ints, double* lambda, double* E, double* dEdC,
                            double* dEdn, double* max_asym_out, double* J, double* K) {
  if (!ctx) return fail(nullptr, PNOF_E_ARG, "context is NULL");
  pnof_status st = check_problem(ctx, prob);
  if (st != PNOF_OK) return st;
  if ((st = check_ptrs(ctx, {C, n, H, ints, lambda, E}, "pnof_lagrangian")) != PNOF_OK) return st;
  if ((st = check_ctx(ctx)) != PNOF_OK) return st;
  Req r;
  r.lam = lambda;
  r.E = E;
  r.dEdC = dEdC;
  r.dEdn = dEdn;
  r.asym = max_asym_out;
  r.J = J;
  r.K = K;
  r.need_y = true;
  r.need_e = true;
  return run_step(ctx, prob, C, n, H, ints, r);
}

pnof_status pnof_lagrangian_noalloc(pnof_ctx ctx, const pnof_problem* prob, const double* C, const double* n,
                                    const double* H, const void* ints, double* lambda, double* E, double* dEdC,
                                    double* dEdn, double* max_asym_out, double* J, double* K) {
  if (!ctx) return fail(nullptr, PNOF_E_ARG, "context is NULL");
  pnof_status st = check_problem(ctx, prob);
  if (st != PNOF_OK) return st;
  if ((st = check_ptrs(ctx, {C, n, H, ints, lambda, E}, "pnof_lagrangian_noalloc")) != PNOF_OK) return st;
  if ((st = check_ctx(ctx)) != PNOF_OK) return st;
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (ctx->device < kMaxDevices) ws = g_scratch[ctx->device];
  }
  if (!ws) return fail(ctx, PNOF_E_DEVICE, "the static workspace of this device was not set up");
  Req r;
  r.lam = lambda;
  r.E = E;
  r.dEdC = dEdC;
  r.dEdn = dEdn;
  r.asym = max_asym_out;
  r.J = J;
  r.K = K;
  r.need_y = true;
  r.need_e = true;
  r.ws = static_cast<char*>(ws);
  r.ws_bytes = PNOF_STATIC_SCRATCH_BYTES;
  r.one_stream = true;
  return run_step(ctx, prob, C, n, H, ints, r);
}

namespace {
// Symmetric float64 eigensolver: A (n x n, symmetric, row-major; destroyed) -> ascending eigenvalues
// w and eigenvectors U (column-major).  The Householder reduction runs on the library's kernels
// (k_eig.hip), A = Q T Q^T.  The library's divide-and-conquer solver (k_tridiag.hip) solves the
// tridiagonal problem, eigenvectors Z into A's storage, while the context's second stream forms
// Q = H_0 ... H_{n-2} explicitly (reflectors applied to the identity in blocks, k_eig.hip
// form_q_f64); then U = Q Z.  Sizes outside [3, TRIDIAG_MAX_N] take rocSOLVER's dsyevd.  info
// (device) receives the solver's status (0 = converged).
struct EighWs {
  double* Vh = nullptr;    // n * n
  double* p2 = nullptr;    // 2n
  double* e = nullptr;     // n
  double* tau = nullptr;   // n
  double* T = nullptr;     // form_q_ws_doubles(n): Q's formation
  double* Q = nullptr;     // n * n
  double* dc = nullptr;    // tridiag_dc_ws_doubles(n): the tridiagonal eigensolver's workspace
};
EighWs take_eigh_ws(Arena& a, int n) {
  EighWs w;
  w.Vh = a.take<double>((long long)n * n);
  w.p2 = a.take<double>(2LL * n);
  w.e = a.take<double>(n);
  w.tau = a.take<double>(n);
  w.T = a.take<double>(form_q_ws_doubles(std::max(n, 3)));
  w.Q = a.take<double>((long long)n * n);
  w.dc = a.take<double>(tridiag_dc_ws_doubles(std::max(n, 1)));
  return w;
}
pnof_status eigh(pnof_ctx ctx, int n, double* A, double* w, double* U, const EighWs& ws, int* info) {
  hipStream_t s = ctx->stream;
  if (n < 3 || n > TRIDIAG_MAX_N) {
    rocblas_status rs = rocsolver_dsyevd(ctx->blas, rocblas_evect_original, rocblas_fill_upper, n, A, n, w, ws.e, info);
    if (rs != rocblas_status_success) return fail(ctx, PNOF_E_DEVICE, "rocsolver_dsyevd failed to launch");
    DEV_CHECK(ctx, hipMemcpyAsync(U, A, sizeof(double) * n * n, hipMemcpyDeviceToDevice, s));
    return PNOF_OK;
  }
  if (!ws.Vh || !ws.p2 || !ws.e || !ws.tau || !ws.T || !ws.Q || !ws.dc)
    return fail(ctx, PNOF_E_ARG, "eigensolver workspace missing");
  RB_CHECK(ensure_aux(ctx));
  DEV_CHECK(ctx, tridiag_f64(s, n, A, ws.Vh, ws.p2, w, ws.e, ws.tau));
  DEV_CHECK(ctx, hipEventRecord(ctx->fork_ev, s));
  DEV_CHECK(ctx, hipStreamWaitEvent(ctx->aux, ctx->fork_ev, 0));
  DEV_CHECK(ctx, form_q_f64(ctx->aux, n, ws.Vh, ws.tau, ws.T, ws.Q));
  DEV_CHECK(ctx, hipEventRecord(ctx->join_ev, ctx->aux));
  double* Z = A;   // free after the reduction
  const hipError_t de = tridiag_eig_dc(s, n, w, ws.e, Z, ws.dc, info);
  DEV_CHECK(ctx, hipStreamWaitEvent(s, ctx->join_ev, 0));   // joined on every path: Q uses the workspace
  DEV_CHECK(ctx, de);
  // U = Q Z, all column-major
  RB_CHECK(dprod(ctx, n, n, n, ws.Q, 1, n, Z, 1, n, U, 1, n));
  return PNOF_OK;
}
}  // namespace

pnof_status pnof_orbital_step(pnof_ctx ctx, int32_t nbf, const double* lambda, const double* C,
                              const double* diag_prev, double zeta, double* C_new, double* eps, double* S_out) {
  if (!ctx) return fail(nullptr, PNOF_E_ARG, "context is NULL");
  if (nbf <= 0) return fail(ctx, PNOF_E_SHAPE, "nbf must be positive");
  if (!std::isfinite(zeta)) return fail(ctx, PNOF_E_ARG, "zeta must be finite");
  pnof_status st = check_ptrs(ctx, {lambda, C, C_new, eps}, "pnof_orbital_step");
  if (st != PNOF_OK) return st;
  if (C_new == C || C_new == lambda) return fail(ctx, PNOF_E_ARG, "C_new must not alias C or lambda");
  if ((st = check_ctx(ctx)) != PNOF_OK) return st;
  const long long n2 = (long long)nbf * nbf;
  Arena probe(nullptr);
  probe.take<double>(n2);
  probe.take<double>(n2);
  take_eigh_ws(probe, nbf);
  probe.take<int>(4);
  char* ws = nullptr;
  if ((st = get_ws(ctx, probe.off + 256, &ws)) != PNOF_OK) return st;
  Arena a(ws);
  double* A = a.take<double>(n2);
  double* U = a.take<double>(n2);
  const EighWs ew = take_eigh_ws(a, nbf);
  int* info = a.take<int>(4);
  hipStream_t s = ctx->stream;
  DEV_CHECK(ctx, build_s(s, nbf, lambda, diag_prev, zeta, A));
  if (S_out) DEV_CHECK(ctx, hipMemcpyAsync(S_out, A, n2 * sizeof(double), hipMemcpyDeviceToDevice, s));
  {
    StageTimer t_(ctx, PNOF_STAGE_EIG);
    if ((st = eigh(ctx, nbf, A, eps, U, ew, info)) != PNOF_OK) return st;
  }
  DEV_CHECK(ctx, sign_fix_cols(s, nbf, U));
  // C_new[mu][j] = sum_i C[mu][i] U[i][j], U column-major: U[i][j] = U[j*nbf + i]
  RB_CHECK(dprod(ctx, nbf, nbf, nbf, C, nbf, 1, U, 1, nbf, C_new, nbf, 1));
  DEV_CHECK(ctx, hipMemcpyAsync(ctx->host_info, info, sizeof(int), hipMemcpyDeviceToHost, s));
  DEV_CHECK(ctx, hipStreamSynchronize(s));
  if (*ctx->host_info != 0)
    return fail(ctx, PNOF_E_EIG, "eigensolver did not converge (info = " + std::to_string(*ctx->host_info) + ")");
  return PNOF_OK;
}

pnof_status pnof_nofmp2_terms(pnof_ctx ctx, const pnof_problem* prob, const double* C, const double* n,
                              const double* H, const void* ints, double* E_hf, double* E_sta) {
  pnof_status st = check_ctx(ctx);
  if (st != PNOF_OK) return st;
  if ((st = check_problem(ctx, prob)) != PNOF_OK) return st;
  if ((st = check_ptrs(ctx, {C, n, H, ints, E_hf, E_sta}, "pnof_nofmp2_terms")) != PNOF_OK) return st;
  const int nact = prob->npairs * (prob->ncwo + 1) + prob->nsingle;
  DevBuf db(ctx);
  double* J = db.get<double>((long long)nact * nact);
  double* K = db.get<double>((long long)nact * nact);
  double* Hpp = db.get<double>(nact);
  double* partials = db.get<double>(256);
  if (!db.ok) return fail(ctx, PNOF_E_NOMEM, "allocation failed");
  Req r;
  r.J = J;
  r.K = K;
  r.Hpp = Hpp;
  if ((st = run_step(ctx, prob, C, nullptr, H, ints, r)) != PNOF_OK) return st;
  DEV_CHECK(ctx, nofmp2_terms(ctx->stream, nact, prob->npairs, prob->ncwo, prob->nsingle, n, Hpp, J, K, partials, E_hf,
                              E_sta));
  return PNOF_OK;
}

pnof_status pnof_optimize_on(pnof_ctx ctx, const pnof_problem* prob, int32_t kind, const double* C,
                             const double* H, const double* J, const double* K, double* gamma,
                             const pnof_on_opts* opts, double* E, int32_t* iterations) {
  pnof_status st = check_ctx(ctx);
  if (st != PNOF_OK) return st;
  if ((st = check_problem(ctx, prob)) != PNOF_OK) return st;
  if (kind != 0 && kind != 1) return fail(ctx, PNOF_E_ARG, "kind must be 0 (sigmoid) or 1 (trigonometric)");
  if ((st = check_ptrs(ctx, {C, H, J, K, gamma, E}, "pnof_optimize_on")) != PNOF_OK) return st;
  const int nbf = prob->nbf, nact = prob->npairs * (prob->ncwo + 1) + prob->nsingle;
  DevBuf db(ctx);
  double* HC = db.get<double>((long long)nbf * nact);
  double* Hpp = db.get<double>(nact);
  if (!db.ok) return fail(ctx, PNOF_E_NOMEM, "allocation failed");
  if ((st = hpp_of(ctx, nbf, nact, C, H, HC, Hpp)) != PNOF_OK) return st;
  OnObjective o;
  if ((st = on_objective_init(ctx, db, prob, kind, Hpp, J, K, o)) != PNOF_OK) return st;
  std::vector<double> x(o.ngam);
  DEV_CHECK(ctx, hipMemcpyAsync(x.data(), gamma, sizeof(double) * o.ngam, hipMemcpyDeviceToHost, ctx->stream));
  DEV_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  pnof_on_opts op = opts ? *opts : pnof_on_opts{0, 0, 0.0};
  double f = 0.0;
  int it = 0;
  if ((st = lbfgs(o, x, op, f, it)) != PNOF_OK) return st;
  DEV_CHECK(ctx, hipMemcpyAsync(gamma, x.data(), sizeof(double) * o.ngam, hipMemcpyHostToDevice, ctx->stream));
  DEV_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  *E = f;
  if (iterations) *iterations = it;
  return PNOF_OK;
}

pnof_status pnof_optimize(pnof_ctx ctx, const pnof_problem* prob, const double* H, const void* ints,
                          double* C, double* gamma, double* n, const pnof_opt_opts* opts,
                          pnof_opt_result* result) {
  pnof_status st = check_ctx(ctx);
  if (st != PNOF_OK) return st;
  if ((st = check_problem(ctx, prob)) != PNOF_OK) return st;
  if (!opts || !result) return fail(ctx, PNOF_E_ARG, "opts and result are required");
  const pnof_opt_opts op = *opts;
  if ((st = check_ptrs(ctx, {H, ints, C, n}, "pnof_optimize")) != PNOF_OK) return st;
  if (!op.fix_n && !gamma) return fail(ctx, PNOF_E_ARG, "gamma is required unless fix_n");
  if (op.on_kind != 0 && op.on_kind != 1) return fail(ctx, PNOF_E_ARG, "on_kind must be 0 or 1");
  const int nbf = prob->nbf, nact = prob->npairs * (prob->ncwo + 1) + prob->nsingle;
  const long long nn = (long long)nbf * nbf, n2 = (long long)nact * nact;
  const int maxit = op.maxit > 0 ? op.maxit : 200;
  const int ndiis = op.ndiis > 1 ? op.ndiis : 0;
  hipStream_t s = ctx->stream;
  DevBuf db(ctx);
  double* lam = db.get<double>(nn);
  double* S = db.get<double>(nn);
  double* Cn = db.get<double>(nn);
  double* T1 = db.get<double>(nn);
  double* diag = db.get<double>(nbf);
  double* Ueig = db.get<double>(nn);
  EighWs ew;
  ew.Vh = db.get<double>(nn);
  ew.p2 = db.get<double>(2LL * nbf);
  ew.e = db.get<double>(nbf);
  ew.tau = db.get<double>(nbf);
  ew.T = db.get<double>(form_q_ws_doubles(std::max(nbf, 3)));
  ew.Q = db.get<double>(nn);
  ew.dc = db.get<double>(tridiag_dc_ws_doubles(nbf));
  int* info = db.get<int>(4);
  double* J = db.get<double>(n2);
  double* K = db.get<double>(n2);
  double* Hpp = db.get<double>(nact);
  double* scal = db.get<double>(4);   // E, max_asym
  std::vector<double*> Fao(ndiis), Eao(ndiis);
  for (int i = 0; i < ndiis; ++i) {
    Fao[i] = db.get<double>(nn);
    Eao[i] = db.get<double>(nn);
  }
  if (!db.ok) return fail(ctx, PNOF_E_NOMEM, "allocation of the optimisation buffers failed");
  OnObjective o;
  if ((st = on_objective_init(ctx, db, prob, op.on_kind, Hpp, J, K, o)) != PNOF_OK) return st;
  std::vector<double> gam;
  if (!op.fix_n) {
    gam.resize(o.ngam);
    DEV_CHECK(ctx, hipMemcpyAsync(gam.data(), gamma, sizeof(double) * o.ngam, hipMemcpyDeviceToHost, s));
    DEV_CHECK(ctx, hipStreamSynchronize(s));
  }
  pnof_problem pr = *prob;
  pr.flags = 0;
  double host2[2];
  // E (and lambda, its asymmetry) of (C, n)
  auto lagr = [&](double& E, double& asym) -> pnof_status {
    Req r;
    r.lam = lam;
    r.E = scal;
    r.asym = scal + 1;
    r.need_y = r.need_e = true;
    pnof_status st2 = run_step(ctx, &pr, C, n, H, ints, r);
    if (st2 != PNOF_OK) return st2;
    DEV_CHECK(ctx, hipMemcpyAsync(host2, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    DEV_CHECK(ctx, hipStreamSynchronize(s));
    E = host2[0];
    asym = host2[1];
    return PNOF_OK;
  };
  // occupations for the current orbitals (Section 3.1): returns E[n^{j+1}, phi^j]
  auto occupations = [&](double& En) -> pnof_status {
    Req r;
    r.J = J;
    r.K = K;
    r.Hpp = Hpp;
    pnof_status st2 = run_step(ctx, &pr, C, nullptr, H, ints, r);
    if (st2 != PNOF_OK) return st2;
    if (op.fix_n) {
      DEV_CHECK(ctx, coeffs(s, nact, pr.npairs, pr.ncwo, pr.nsingle, pr.functional, n, o.alpha, o.beta, nullptr));
      DEV_CHECK(ctx, energy(s, nbf, nact, n, Hpp, o.alpha, o.beta, J, K, nullptr, nullptr, nullptr, nullptr, nullptr,
                            0, 0, o.partials, o.E));
      DEV_CHECK(ctx, hipMemcpyAsync(host2, o.E, sizeof(double), hipMemcpyDeviceToHost, s));
      DEV_CHECK(ctx, hipStreamSynchronize(s));
      En = host2[0];
      return PNOF_OK;
    }
    int it = 0;
    st2 = lbfgs(o, gam, op.on, En, it);
    if (st2 != PNOF_OK) return st2;
    DEV_CHECK(ctx, hipMemcpyAsync(gamma, gam.data(), sizeof(double) * o.ngam, hipMemcpyHostToDevice, s));
    DEV_CHECK(ctx, on_map(s, op.on_kind, pr.npairs, pr.ncwo, pr.nsingle, gamma, n, nullptr));
    return PNOF_OK;
  };
  // diagonalise S (overwritten by the eigenvectors), new diagonal, C <- C U
  auto diagonalise = [&]() -> pnof_status {
    pnof_status se = eigh(ctx, nbf, S, diag, Ueig, ew, info);
    if (se != PNOF_OK) return se;
    DEV_CHECK(ctx, sign_fix_cols(s, nbf, Ueig));
    DEV_CHECK(ctx, gemm_f64(s, nbf, nbf, nbf, 1, 1.0, C, nbf, 1, 0, Ueig, 1, nbf, 0, 0.0, Cn, nbf, 1, 0));
    DEV_CHECK(ctx, hipMemcpyAsync(C, Cn, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
    int hinfo = 0;
    DEV_CHECK(ctx, hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, s));
    DEV_CHECK(ctx, hipStreamSynchronize(s));
    if (hinfo != 0) return fail(ctx, PNOF_E_EIG, "eigensolver did not converge");
    return PNOF_OK;
  };
  // initial step
  double En = 0.0, E0 = 0.0, asym = 0.0, Eprev = 0.0;
  if ((st = occupations(En)) != PNOF_OK) return st;
  if ((st = lagr(E0, asym)) != PNOF_OK) return st;
  DEV_CHECK(ctx, build_s(s, nbf, lam, nullptr, 0.0, S));
  if ((st = diagonalise()) != PNOF_OK) return st;
  if ((st = lagr(Eprev, asym)) != PNOF_OK) return st;
  pnof_opt_result res{};
  res.E = Eprev;
  res.max_asym = asym;
  int nstored = 0, head = 0;
  int it = 0;
  for (it = 1; it <= maxit; ++it) {
    if ((st = occupations(En)) != PNOF_OK) return st;
    double Efix = 0.0, Enew = 0.0;
    if ((st = lagr(Efix, asym)) != PNOF_OK) return st;
    DEV_CHECK(ctx, build_s(s, nbf, lam, diag, op.zeta, S));
    if (ndiis) {
      // store F_AO = C F C^T and e_AO = C offdiag(F) C^T; combine when two or more are stored
      DEV_CHECK(ctx, gemm_f64(s, nbf, nbf, nbf, 1, 1.0, C, nbf, 1, 0, S, nbf, 1, 0, 0.0, T1, nbf, 1, 0));
      DEV_CHECK(ctx, gemm_f64(s, nbf, nbf, nbf, 1, 1.0, T1, nbf, 1, 0, C, 1, nbf, 0, 0.0, Fao[head], nbf, 1, 0));
      DEV_CHECK(ctx, offdiag_copy(s, nbf, S, Cn));
      DEV_CHECK(ctx, gemm_f64(s, nbf, nbf, nbf, 1, 1.0, C, nbf, 1, 0, Cn, nbf, 1, 0, 0.0, T1, nbf, 1, 0));
      DEV_CHECK(ctx, gemm_f64(s, nbf, nbf, nbf, 1, 1.0, T1, nbf, 1, 0, C, 1, nbf, 0, 0.0, Eao[head], nbf, 1, 0));
      head = (head + 1) % ndiis;
      nstored = std::min(nstored + 1, ndiis);
      if (nstored >= 2) {
        const int m = nstored;
        std::vector<double> A((m + 1) * (m + 1), 0.0), rhs(m + 1, 0.0);
        rocblas_set_pointer_mode(ctx->blas, rocblas_pointer_mode_host);
        for (int i = 0; i < m; ++i)
          for (int j = 0; j <= i; ++j) {
            double v = 0.0;
            if (rocblas_ddot(ctx->blas, (int)nn, Eao[i], 1, Eao[j], 1, &v) != rocblas_status_success)
              return fail(ctx, PNOF_E_DEVICE, "rocblas_ddot failed");
            A[i * (m + 1) + j] = A[j * (m + 1) + i] = v;
          }
        for (int i = 0; i < m; ++i) A[i * (m + 1) + m] = A[m * (m + 1) + i] = -1.0;
        rhs[m] = -1.0;
        if (solve_small(A, rhs, m + 1)) {
          DEV_CHECK(ctx, fill_f64(s, Cn, nn, 0.0));
          for (int i = 0; i < m; ++i) {
            const double c = rhs[i];
            if (rocblas_daxpy(ctx->blas, (int)nn, &c, Fao[i], 1, Cn, 1) != rocblas_status_success)
              return fail(ctx, PNOF_E_DEVICE, "rocblas_daxpy failed");
          }
          // S = C^T F_AO C
          DEV_CHECK(ctx, gemm_f64(s, nbf, nbf, nbf, 1, 1.0, Cn, nbf, 1, 0, C, nbf, 1, 0, 0.0, T1, nbf, 1, 0));
          DEV_CHECK(ctx, gemm_f64(s, nbf, nbf, nbf, 1, 1.0, C, 1, nbf, 0, T1, nbf, 1, 0, 0.0, S, nbf, 1, 0));
        }
      }
    }
    if ((st = diagonalise()) != PNOF_OK) return st;
    if ((st = lagr(Enew, asym)) != PNOF_OK) return st;
    res.d_n = std::fabs(En - Eprev);
    res.d_phi = std::fabs(Enew - Efix);
    res.d_E = std::fabs(Enew - Eprev);
    res.max_asym = asym;
    res.E = Enew;
    Eprev = Enew;
    if (asym < op.delta) {
      res.converged = 1;
      break;
    }
    if (res.d_n < op.eps_n && res.d_phi < op.eps_phi && res.d_E < op.eps) break;
  }
  res.iterations = std::min(it, maxit);
  *result = res;
  return PNOF_OK;
}

pnof_status pnof_batch_plan(pnof_ctx ctx, int32_t ninst, const pnof_problem* probs, pnof_batch* out) {
  if (!out) return fail(ctx, PNOF_E_ARG, "output pointer is NULL");
  *out = nullptr;
  pnof_status st = check_ctx(ctx);
  if (st != PNOF_OK) return st;
  if (ninst <= 0 || !probs) return fail(ctx, PNOF_E_ARG, "a batch needs ninst > 0 problems");
  const int prec = probs[0].precision;
  for (int i = 0; i < ninst; ++i) {
    if ((st = check_problem(ctx, &probs[i])) != PNOF_OK)
      return fail(ctx, st, "instance " + std::to_string(i) + ": " + ctx->err);
    if (probs[i].ints != PNOF_INTS_DF_BF16)
      return fail(ctx, PNOF_E_UNSUPPORTED, "batches take bfloat16 density-fitting factors (PNOF_INTS_DF_BF16)");
    if (probs[i].precision != PNOF_BF16_SPLIT && probs[i].precision != PNOF_BF16)
      return fail(ctx, PNOF_E_UNSUPPORTED, "batches run the bf16 contractions (PNOF_BF16_SPLIT or PNOF_BF16)");
    if (probs[i].precision != prec) return fail(ctx, PNOF_E_ARG, "all instances of a batch share one precision");
    if (probs[i].flags != 0) return fail(ctx, PNOF_E_UNSUPPORTED, "batches take no flags");
  }
  int khz = 0, nxcc = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess || khz <= 0) {
    hipGetLastError();
    return fail(ctx, PNOF_E_DEVICE, "the device wall-clock rate is unavailable");
  }
  if (hipDeviceGetAttribute(&nxcc, hipDeviceAttributeNumberOfXccs, ctx->device) != hipSuccess || nxcc <= 0) {
    hipGetLastError();
    nxcc = 1;   // one group: every instance on whichever die runs the first block
  }
  nxcc = std::min(nxcc, PERSIST_MAX_DIES);
  pnof_batch b = new pnof_batch_s();
  b->ctx = ctx;
  b->ninst = ninst;
  b->clock_khz = (double)khz;
  b->ps.ndie = b->dev_dies = nxcc;
  b->terms = prec == PNOF_BF16_SPLIT ? 3 : 1;
  // the split mode adds the two launches of the scale bounds; the last one forms dE/dgamma
  b->launches = b->terms > 1 ? 16 : 14;
  b->probs.assign(probs, probs + ninst);
  b->inst.resize(ninst);
  // carve (measure, then allocate and carve again)
  auto carve_all = [&](char* base) -> size_t {
    Arena a(base);
    b->geo.clear();
    for (int i = 0; i < ninst; ++i) {
      const pnof_problem& p = probs[i];
      const BatchGeom g = batch_geom(p);
      b->geo.push_back(g);
      BInst& d = b->inst[i];
      d = BInst{};
      d.nbf = g.nbf; d.nact = g.nact; d.naux = g.naux; d.npairs = p.npairs; d.ncwo = p.ncwo; d.nsingle = p.nsingle;
      d.functional = p.functional; d.terms = b->terms;
      d.ldk = g.ldk; d.ldw = g.ldw; d.nact32 = g.nact32; d.ns2 = g.ns2; d.ns3 = g.ns3;
      const long long n2 = (long long)g.nact * g.nact, ny = (long long)g.nbf * g.nact;
      d.Bp = a.take<u16>((long long)g.naux * g.nbf * g.ldk);
      d.cth = a.take<u16>((long long)g.nact32 * g.ldk);
      d.xth = a.take<u16>((long long)g.naux * g.nact32 * g.ldk);
      d.wh = a.take<u16>((long long)g.naux * g.nact32 * g.ldw);
      if (b->terms > 1) {
        d.ctl = a.take<u16>((long long)g.nact32 * g.ldk);
        d.ch16 = a.take<u16>((long long)g.nact32 * g.ldk);
        d.cl16 = a.take<u16>((long long)g.nact32 * g.ldk);
        d.xtl = a.take<u16>((long long)g.naux * g.nact32 * g.ldk);
        d.wl = a.take<u16>((long long)g.naux * g.nact32 * g.ldw);
        d.bnd = a.take<uint32_t>(SCL_CALL + 2);
        d.colb = a.take<float>(4LL * g.nact);
      }
      d.alpha = a.take<double>(n2);
      d.beta = a.take<double>(n2);
      d.beta32 = a.take<float>(n2);
      d.J = a.take<double>(n2);
      d.K = a.take<double>(n2);
      d.Kpart = a.take<double>((long long)g.ns2 * n2);
      d.HC = a.take<double>(ny);
      d.Y2e = a.take<double>(ny);
      d.Y = a.take<double>(ny);
      d.Ypart = a.take<float>((long long)g.ns3 * ny);
      d.Hpp = a.take<double>(g.nact);
      d.D = a.take<double>((long long)g.naux * g.nact);
      d.dbuf = a.take<double>((long long)g.naux * g.nact);
      d.epart = a.take<double>(BATCH_EPARTS);
    }
    b->d_inst = a.take<BInst>(ninst);
    b->d_g1 = a.take<G1Args>(ninst);
    b->d_g2 = a.take<G2Args>(ninst);
    b->d_g3 = a.take<G3Args>(ninst);
    b->d_off = a.take<int>(3LL * (ninst + 1));
    b->d_f64 = a.take<F64Gemm>(4LL * ninst);
    b->d_cnt = a.take<int>((long long)ninst * PH_N);
    b->ps.cnt = b->d_cnt;
    b->ps.claim = a.take<int>((long long)ninst * PH_N);
    b->ps.done = a.take<int>((long long)ninst * PH_N);
    b->ps.phase = a.take<int>(ninst);
    b->ps.t_end = a.take<unsigned long long>(ninst);
    b->ps.t_start = a.take<unsigned long long>(1);
    b->ps.prog = a.take<int>(4);
    b->d_order = a.take<int>(ninst);
    b->d_xoff = a.take<int>(PERSIST_MAX_DIES + 1);
    b->ps.order = b->d_order;
    b->ps.xoff = b->d_xoff;
    b->ps.die_of = a.take<int>(PERSIST_MAX_DIES);
    return a.off + 256;
  };
  for (int i = 0; i < ninst; ++i) {
    const BatchGeom g = batch_geom(probs[i]);
    const long long lim = (1LL << 31) - 1;
    if (2LL * g.naux * g.nbf * g.ldk > lim || 2LL * g.naux * g.nact32 * g.ldk > lim || 2LL * g.naux * g.nact32 * g.ldw > lim) {
      delete b;
      return fail(ctx, PNOF_E_UNSUPPORTED, "instance " + std::to_string(i) + " is too large for a batch (2 GiB per buffer)");
    }
  }
  b->bytes = carve_all(nullptr);
  if (hipMalloc(&b->ws, b->bytes) != hipSuccess) {
    hipGetLastError();
    delete b;
    return fail(ctx, PNOF_E_NOMEM, "batch workspace allocation failed");
  }
  carve_all(b->ws);
  // grid maxima and work-item offsets
  std::vector<int> off(3 * (ninst + 1), 0);
  BMax mx{};
  for (int i = 0; i < ninst; ++i) {
    const BatchGeom& g = b->geo[i];
    const long long n2 = (long long)g.nact * g.nact, ny = (long long)g.nbf * g.nact;
    mx.nbf = std::max(mx.nbf, g.nbf);
    mx.nact = std::max(mx.nact, g.nact);
    mx.pack = std::max(mx.pack, (long long)g.naux * g.nact32 * g.ldk + (long long)g.naux * g.nbf * g.ldk);
    mx.prep = std::max(mx.prep, std::max(n2, (long long)g.nact * g.nbf));
    mx.y = std::max(mx.y, ny);
    mx.k = std::max(mx.k, n2);
    mx.diag = std::max(mx.diag, (long long)g.naux * g.nact);
    mx.rows = std::max(mx.rows, (long long)g.naux * g.nbf);
    b->maxM[0] = std::max(b->maxM[0], g.nbf);  b->maxN[0] = std::max(b->maxN[0], g.nact);   // H C_A
    b->maxM[1] = std::max(b->maxM[1], g.naux); b->maxN[1] = std::max(b->maxN[1], g.nact);   // D alpha
    b->maxM[2] = std::max(b->maxM[2], g.nact); b->maxN[2] = std::max(b->maxN[2], g.nact);   // D^T D
    b->maxM[3] = std::max(b->maxM[3], g.nbf);  b->maxN[3] = std::max(b->maxN[3], g.nact);   // C^T Y
  }
  b->mx = mx;
  batch_resolve_tiles(b);
  *out = b;
  return PNOF_OK;
}

pnof_status pnof_batch_set_tiles(pnof_batch b, int32_t x_tile, int32_t b_tile, int32_t y_tile) {
  if (!b) return fail(nullptr, PNOF_E_ARG, "batch is NULL");
  pnof_ctx ctx = b->ctx;
  pnof_status st = check_ctx(ctx);
  if (st != PNOF_OK) return st;
  const int v[3] = {x_tile, b_tile, y_tile};
  for (int k = 0; k < 3; ++k)
    if (v[k] != 0 && v[k] != 64 && v[k] != 128) return fail(ctx, PNOF_E_ARG, "tile widths are 0 (automatic), 64 or 128");
  for (int k = 0; k < 3; ++k) b->req[k] = v[k];
  batch_resolve_tiles(b);
  batch_drop_graph(b);
  if (b->bound) DEV_CHECK(ctx, batch_offsets(b, ctx->stream));
  return PNOF_OK;
}

pnof_status pnof_batch_get_tiles(pnof_batch b, int32_t* tiles) {
  if (!b) return fail(nullptr, PNOF_E_ARG, "batch is NULL");
  if (!tiles) return fail(b->ctx, PNOF_E_ARG, "tiles is NULL");
  for (int k = 0; k < 3; ++k) tiles[k] = b->tile[k];
  return PNOF_OK;
}

pnof_status pnof_batch_bind(pnof_batch b, const pnof_batch_io* io) {
  if (!b) return fail(nullptr, PNOF_E_ARG, "batch is NULL");
  pnof_ctx ctx = b->ctx;
  pnof_status st = check_ctx(ctx);
  if (st != PNOF_OK) return st;
  if (!io) return fail(ctx, PNOF_E_ARG, "io is NULL");
  const int n = b->ninst;
  for (int i = 0; i < n; ++i)
    if (!io[i].C || !io[i].n || !io[i].H || !io[i].ints || !io[i].lambda || !io[i].E)
      return fail(ctx, PNOF_E_ARG, "instance " + std::to_string(i) + ": C, n, H, ints, lambda and E are required");
  for (int i = 0; i < n; ++i) {
    if (io[i].dEdgamma && (!io[i].gamma || !io[i].dEdn))
      return fail(ctx, PNOF_E_ARG, "instance " + std::to_string(i) + ": dEdgamma needs gamma and dEdn");
    if (io[i].gamma && io[i].on_kind != 0 && io[i].on_kind != 1)
      return fail(ctx, PNOF_E_ARG, "instance " + std::to_string(i) + ": on_kind is 0 (sigmoid) or 1 (trigonometric)");
  }
  batch_drop_graph(b);
  std::vector<G1Args> g1(n);
  std::vector<G2Args> g2(n);
  std::vector<G3Args> g3(n);
  std::vector<F64Gemm> f(4 * n);
  for (int i = 0; i < n; ++i) {
    BInst& d = b->inst[i];
    const BatchGeom& g = b->geo[i];
    d.C = io[i].C; d.n = io[i].n; d.H = io[i].H; d.B = static_cast<const u16*>(io[i].ints);
    d.lam = io[i].lambda; d.E = io[i].E; d.dEdC = io[i].dEdC; d.dEdn = io[i].dEdn; d.asym = io[i].max_asym;
    d.gamma = io[i].gamma; d.dEdgamma = io[i].dEdgamma; d.on_kind = io[i].on_kind;
    const long long nct = (long long)g.nact32 * g.ldk, nxt = (long long)g.naux * g.nact32 * g.ldk,
                    nw = (long long)g.naux * g.nact32 * g.ldw;
    const WsDims wd{g.nact32, 2 * nct, 2 * nxt, 2 * nw};
    // X: the compact bf16 pair of C (or one bf16 value) times B; b: the fp16 pair of C~ sC in the
    // split mode; the scales of each instance come from its bound words (one chunk: all of B)
    g1[i] = G1Args{g.nbf, g.nact, g.naux, d.cth, d.ctl, g.ldk, d.Bp, nullptr, (long long)g.nbf * g.ldk, g.ldk,
                   2LL * g.naux * g.nbf * g.ldk, d.xth, d.xtl, g.ldk, wd, d.bnd, 0};
    const u16* c2h = b->terms > 1 ? d.ch16 : d.cth;
    const u16* c2l = b->terms > 1 ? d.cl16 : nullptr;
    g2[i] = G2Args{g.nbf, g.nact, g.naux, g.ns2, c2h, c2l, g.ldk, d.xth, d.xtl, g.ldk, d.beta32, d.Kpart, d.D,
                   d.wh, d.wl, g.ldw, wd, d.bnd, 0};
    g3[i] = G3Args{g.nbf, g.nact, g.naux, g.ns3, d.xth, d.xtl, g.ldk, d.wh, d.wl, g.ldw, d.Ypart, wd, d.bnd, 0};
    f[i] = F64Gemm{g.nbf, g.nact, g.nbf, 1.0, d.H, g.nbf, 1, d.C, g.nbf, 1, 0.0, d.HC, g.nact, 1};
    f[n + i] = F64Gemm{g.naux, g.nact, g.nact, 1.0, d.D, g.nact, 1, d.alpha, g.nact, 1, 0.0, d.dbuf, g.nact, 1};
    f[2 * n + i] = F64Gemm{g.nact, g.nact, g.naux, 1.0, d.D, 1, g.nact, d.D, g.nact, 1, 0.0, d.J, g.nact, 1};
    f[3 * n + i] = F64Gemm{g.nbf, g.nact, g.nbf, 1.0, d.C, 1, g.nbf, d.Y, g.nact, 1, 0.0, d.lam, g.nbf, 1};
  }
  hipStream_t s = ctx->stream;
  DEV_CHECK(ctx, hipMemcpyAsync(b->d_inst, b->inst.data(), sizeof(BInst) * n, hipMemcpyHostToDevice, s));
  DEV_CHECK(ctx, hipMemcpyAsync(b->d_g1, g1.data(), sizeof(G1Args) * n, hipMemcpyHostToDevice, s));
  DEV_CHECK(ctx, hipMemcpyAsync(b->d_g2, g2.data(), sizeof(G2Args) * n, hipMemcpyHostToDevice, s));
  DEV_CHECK(ctx, hipMemcpyAsync(b->d_g3, g3.data(), sizeof(G3Args) * n, hipMemcpyHostToDevice, s));
  DEV_CHECK(ctx, batch_offsets(b, s));
  DEV_CHECK(ctx, hipMemcpyAsync(b->d_f64, f.data(), sizeof(F64Gemm) * f.size(), hipMemcpyHostToDevice, s));
  DEV_CHECK(ctx, batch_pack(s, n, b->d_inst, b->mx));
  if (b->terms > 1) DEV_CHECK(ctx, batch_b_bounds(s, n, b->d_inst, b->mx));
  // the host staging vectors go out of scope: wait for the copies
  DEV_CHECK(ctx, hipStreamSynchronize(s));
  b->bound = true;
  return PNOF_OK;
}

pnof_status pnof_batch_run(pnof_batch b, int32_t flags) {
  if (!b) return fail(nullptr, PNOF_E_ARG, "batch is NULL");
  pnof_ctx ctx = b->ctx;
  pnof_status st = check_ctx(ctx);
  if (st != PNOF_OK) return st;
  if (!b->bound) return fail(ctx, PNOF_E_ARG, "pnof_batch_bind must be called before pnof_batch_run");
  if (flags & ~(PNOF_BATCH_GRAPH | PNOF_BATCH_PERSISTENT)) return fail(ctx, PNOF_E_ARG, "unknown batch run flags");
  const bool persistent = (flags & PNOF_BATCH_PERSISTENT) != 0, use_graph = (flags & PNOF_BATCH_GRAPH) != 0;
  if (persistent && b->terms != 3)
    return fail(ctx, PNOF_E_UNSUPPORTED, "the persistent batch kernel runs the split precision (PNOF_BF16_SPLIT)");
  if (!persistent) {
    if (!b->side) DEV_CHECK(ctx, hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
    for (hipEvent_t& ev : b->ev)
      if (!ev) DEV_CHECK(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  }
  b->last_flags = flags;
  if (!use_graph) {
    DEV_CHECK(ctx, persistent ? batch_enqueue_persistent(b, ctx->stream) : batch_enqueue(b, ctx->stream));
    return PNOF_OK;
  }
  hipGraph_t& graph = persistent ? b->pgraph : b->graph;
  hipGraphExec_t& exec = persistent ? b->pexec : b->exec;
  if (!exec) {
    if (!b->cap) DEV_CHECK(ctx, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    DEV_CHECK(ctx, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = persistent ? batch_enqueue_persistent(b, b->cap) : batch_enqueue(b, b->cap);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) hipGraphDestroy(g);
      hipGetLastError();
      return fail(ctx, PNOF_E_DEVICE, std::string("graph capture failed: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    graph = g;
    DEV_CHECK(ctx, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  }
  DEV_CHECK(ctx, hipGraphLaunch(exec, ctx->stream));
  return PNOF_OK;
}

pnof_status pnof_batch_times(pnof_batch b, double* us) {
  if (!b) return fail(nullptr, PNOF_E_ARG, "batch is NULL");
  pnof_ctx ctx = b->ctx;
  pnof_status st = check_ctx(ctx);
  if (st != PNOF_OK) return st;
  if (!us) return fail(ctx, PNOF_E_ARG, "us is NULL");
  if (b->last_flags < 0 || !(b->last_flags & PNOF_BATCH_PERSISTENT))
    return fail(ctx, PNOF_E_UNSUPPORTED, "completion times are recorded by persistent runs only");
  const int n = b->ninst;
  std::vector<unsigned long long> t(n + 1);
  int prog[4] = {0, 0, 0, 0};
  DEV_CHECK(ctx, hipMemcpyAsync(t.data(), b->ps.t_end, sizeof(unsigned long long) * n, hipMemcpyDeviceToHost, ctx->stream));
  DEV_CHECK(ctx, hipMemcpyAsync(t.data() + n, b->ps.t_start, sizeof(unsigned long long), hipMemcpyDeviceToHost, ctx->stream));
  DEV_CHECK(ctx, hipMemcpyAsync(prog, b->ps.prog, sizeof(int) * 4, hipMemcpyDeviceToHost, ctx->stream));
  DEV_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  if (prog[2] == 2)
    return fail(ctx, PNOF_E_DEVICE, "the persistent batch run stopped: the device's die ids do not map one to one onto "
                                    "its XCC count; its outputs are incomplete (use the grouped form)");
  if (prog[2] != 0 || prog[1] != n)
    return fail(ctx, PNOF_E_DEVICE, "the persistent batch run stalled (" + std::to_string(prog[1]) + " of " +
                                        std::to_string(n) + " instances completed); its outputs are incomplete");
  for (int i = 0; i < n; ++i) us[i] = (double)(t[i] - t[n]) * 1e3 / b->clock_khz;
  return PNOF_OK;
}

pnof_status pnof_batch_set_dies(pnof_batch b, int32_t dies) {
  if (!b) return fail(nullptr, PNOF_E_ARG, "batch is NULL");
  if (dies < 0 || dies > PERSIST_MAX_DIES)
    return fail(b->ctx, PNOF_E_ARG, "dies must be in [0, " + std::to_string(PERSIST_MAX_DIES) + "]");
  b->ps.ndie = dies > 0 ? dies : b->dev_dies;
  batch_drop_graph(b);
  if (b->bound) DEV_CHECK(b->ctx, batch_offsets(b, b->ctx->stream));
  return PNOF_OK;
}

pnof_status pnof_batch_set_stall(pnof_batch b, double microseconds) {
  if (!b) return fail(nullptr, PNOF_E_ARG, "batch is NULL");
  if (!(microseconds >= 0.0) || microseconds > 1e9) return fail(b->ctx, PNOF_E_ARG, "microseconds must be in [0, 1e9]");
  b->stall_us = microseconds > 0.0 ? microseconds : 1e6;
  batch_drop_graph(b);
  return PNOF_OK;
}

pnof_status pnof_batch_info(pnof_batch b, size_t* bytes, int32_t* launches) {
  if (!b) return fail(nullptr, PNOF_E_ARG, "batch is NULL");
  if (bytes) *bytes = b->bytes;
  if (launches) *launches = b->launches;
  return PNOF_OK;
}

void pnof_batch_destroy(pnof_batch b) {
  if (!b) return;
  hipSetDevice(b->ctx->device);
  hipStreamSynchronize(b->ctx->stream);
  batch_drop_graph(b);
  if (b->cap) hipStreamDestroy(b->cap);
  if (b->side) {
    hipStreamSynchronize(b->side);
    hipStreamDestroy(b->side);
  }
  for (hipEvent_t ev : b->ev)
    if (ev) hipEventDestroy(ev);
  if (b->ws) hipFree(b->ws);
  delete b;
}

}  // extern "C"
