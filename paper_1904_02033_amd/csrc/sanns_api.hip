// C ABI of the homomorphic distance stage (see include/sanns.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/sanns.h"
#include "kernels.h"
#include "launch.h"
#include "params.h"

using namespace sanns;

// Device scratch of sanns_distances_noalloc: one copy per GPU, held until the
// process ends.  Host code never uses the name as an address; each device's
// copy is located once with hipGetSymbolAddress (scratch_for_device).
static __device__ __align__(256) unsigned char scratch[SANNS_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_last_error;

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on `device`, which must be current; looked up
// on the first call for each device.
hipError_t scratch_for_device(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

sanns_status fail(sanns_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define HIP_TRY(expr)                                                             \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      return fail(SANNS_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Cache key of a captured batched launch sequence.
struct GraphKey {
  const void* db;
  uint32_t C, d, Q, M;
  const void* ct_in;
  const void* qids;
  const void* ct_out;
  const void* share;
  const void* ws;
  int qt, ct, lds, n_tiles, table, persist;
  const void* pk;
  uint32_t flood_bits;
  uint32_t key[8];
  bool operator<(const GraphKey& o) const { return std::memcmp(this, &o, sizeof *this) < 0; }
};

}  // namespace

struct sanns_ctx {
  sanns_params p{};
  int device = 0;
  int logN = 0;
  PrimeSet ps{};
  DigitSet ds{};
  bool digit_db = false;  // databases carry the int8 digit form (SANNS_FLAG_DIGIT_DB)
  TwSet tws{};
  DecodeConst dec{};
  uint64_t tone = 0;  // floor(2^64 / t)
  uint64_t* d_tw = nullptr;
  uint32_t* d_err = nullptr;
  void* scratch = nullptr;  // this device's copy of `scratch` (sanns_distances_noalloc)
  int flood_bits_max = 0;   // largest b with 2^b <= Delta / 4 (circuit-private form)
  hipStream_t cap_stream = nullptr;
  std::mutex mu;
  // captured batched sequences, least recently used evicted beyond kMaxGraphs
  struct CachedGraph {
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;  // recorded after each launch; awaited before destruction
    uint64_t last_use = 0;
  };
  std::map<GraphKey, CachedGraph> graphs;
  uint64_t graph_clock = 0;
  // pinned staging for host-built schedules: a ring of buffers, each reused
  // once the copy out of it has completed, so that callers on different
  // streams do not wait for each other's copies
  struct Staging {
    void* buf = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
  };
  Staging staging[4];
  int staging_next = 0;
  // schedule override (0 = automatic)
  int force_qt = 0, force_ct = 0, force_lds = 0, force_persist = 0;
  // per-phase profiling: one event pair per phase and call
  bool profiling = false;
  std::vector<std::vector<std::pair<hipEvent_t, hipEvent_t>>> prof_events;
};

namespace {
void drop_profile_events(sanns_ctx* ctx);
}

namespace {

int log2u(uint32_t x) {
  int l = 0;
  while ((1u << l) < x) ++l;
  return l;
}

const int kDefaultLdsVariant = 22;  // fastest at 1M x 128, 64 queries
const size_t kMaxGraphs = 32;       // cached graph execs per context

const int kLogqCap[] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 27, 54, 109, 218, 438, 881};

sanns_status check_params(const sanns_params* p) {
  if (!p) return fail(SANNS_E_INVALID, "null parameters");
  if (p->N < 16 || p->N > 16384 || (p->N & (p->N - 1)))
    return fail(SANNS_E_INVALID, "N = %u is not a power of two in [16, 16384]", p->N);
  if (p->L < 1 || p->L > SANNS_MAX_LIMBS)
    return fail(SANNS_E_INVALID, "L = %u outside [1, %d]", p->L, SANNS_MAX_LIMBS);
  if (p->t < 2 || p->t >= (1ull << 31))
    return fail(SANNS_E_PARAMS, "t = %llu outside [2, 2^31)", (unsigned long long)p->t);
  for (uint32_t l = 0; l < p->L; ++l) {
    const uint64_t q = p->q[l];
    if (q <= (1ull << 32) || q >= (1ull << 54))
      return fail(SANNS_E_PARAMS, "q[%u] outside (2^32, 2^54)", l);
    if (q % (2ull * p->N) != 1) return fail(SANNS_E_PARAMS, "q[%u] != 1 mod 2N", l);
    if (!host::is_prime(q)) return fail(SANNS_E_PARAMS, "q[%u] is not prime", l);
    for (uint32_t j = 0; j < l; ++j)
      if (p->q[j] == q) return fail(SANNS_E_PARAMS, "q[%u] repeats q[%u]", l, j);
  }
  std::vector<uint64_t> qs(p->q, p->q + p->L);
  const int bits = host::log2q_bits(qs);
  const int logN = log2u(p->N);
  if (!(p->flags & SANNS_FLAG_INSECURE_TEST)) {
    if (logN < 10) return fail(SANNS_E_PARAMS, "N < 1024 needs SANNS_FLAG_INSECURE_TEST");
    if (bits > kLogqCap[logN])
      return fail(SANNS_E_PARAMS, "log2 q = %d exceeds the 128-bit cap %d for N = %u", bits,
                  kLogqCap[logN], p->N);
  }
  return SANNS_OK;
}

// Choose the multiply-accumulate kernel: an LDS-staged variant (lds > 0)
// for a batch of at least two queries against every chunk, otherwise the
// (queries x chunks) register tile qt x ct.  q_per_chunk: mean number of
// queries per chunk of a work list.
bool db_has_digits(const sanns_ctx* ctx, uint32_t d) {
  return ctx->digit_db && mfma_supported(ctx->logN, (int)d);
}

// Whether the matrix-core schedule is expected to beat the vector one for Q
// queries against C chunks of dimension d.  Relative costs per (limb, slot),
// from the kernels' times at Q = 64, C = 123, d = 128: the 64-bit vector
// multiply-accumulate 8.6 ms (scales with Q C d); the matrix-core path's
// digit transpose 1.35 ms (Q Dq), MFMA tiles 2.4 ms (64-row x 64-chunk tiles
// x Dp, 4 of them) and sums transpose 1.25 ms (Q C).
bool mfma_expected_faster(uint32_t Q, uint32_t C, uint32_t d) {
  const double Dp = mfma_padded_d((int)d), Dq = mfma_query_d((int)d);
  const double valu = 8.6 * (double)Q * C * d / (64.0 * 123 * 128);
  const double tiles = (double)((2 * Q + 63) / 64) * ((C + 63) / 64);
  const double mfma = 1.35 * Q * Dq / (64.0 * 128) + 2.4 * tiles * Dp / (4.0 * 128) +
                      1.25 * (double)Q * C / (64.0 * 123);
  return mfma < valu;
}

// Whether an all-pairs (or not) call of Q queries against C chunks runs the
// matrix-core schedule: forced by sanns_set_schedule, or chosen by default on
// a digit database when the cost model predicts it faster.
bool call_uses_mfma(const sanns_ctx* ctx, uint32_t Q, uint32_t C, uint32_t d, bool all_pairs) {
  if (!all_pairs || Q < 2 || !db_has_digits(ctx, d)) return false;
  if (ctx->force_lds > 0) return ctx->force_lds == kMfmaSchedule;
  return mfma_expected_faster(Q, C, d);
}

void choose_shape(const sanns_ctx* ctx, uint32_t Q, uint32_t C, uint32_t d, bool regular,
                  double q_per_chunk, int& qt, int& ct, int& lds) {
  lds = 0;
  if (regular && Q >= 2) {
    if (call_uses_mfma(ctx, Q, C, d, true))
      lds = kMfmaSchedule;
    else
      lds = ctx->force_lds > 0 ? ctx->force_lds : kDefaultLdsVariant;
    if (lds == kMfmaSchedule && !db_has_digits(ctx, d)) lds = kDefaultLdsVariant;
    if (lds != kMfmaSchedule && (int)ctx->p.N % mac_lds_min_n(lds) != 0) lds = 0;
  }
  if (ctx->force_qt > 0) {
    qt = ctx->force_qt;
    ct = ctx->force_ct;
  } else if (Q <= 1 || (!regular && q_per_chunk < 2.0)) {
    // one query, or work lists whose chunks are mostly scanned by a single
    // query (the clustered form's cluster chunks): 1 x 8 measured fastest
    qt = 1;
    ct = 8;
  } else {
    qt = 2;
    ct = 4;
  }
}

// Host-built schedule for an explicit work list: group the outputs by chunk,
// split each chunk's queries into groups of qt, and pack chunks that share a
// query group ct at a time.
std::vector<int32_t> build_tiles(const uint32_t* work, uint32_t M, int qt, int ct,
                                 int* n_tiles) {
  std::map<uint32_t, std::vector<std::pair<uint32_t, uint32_t>>> by_chunk;  // k -> (q, m)
  for (uint32_t m = 0; m < M; ++m) by_chunk[work[2 * m + 1]].push_back({work[2 * m], m});
  std::map<std::vector<uint32_t>, std::vector<std::pair<uint32_t, std::vector<int32_t>>>>
      groups;  // query group -> (chunk, outs)
  for (auto& kv : by_chunk) {
    auto& v = kv.second;
    std::sort(v.begin(), v.end());
    for (size_t s = 0; s < v.size(); s += qt) {
      std::vector<uint32_t> g;
      std::vector<int32_t> outs;
      for (size_t a = s; a < std::min(v.size(), s + qt); ++a) {
        g.push_back(v[a].first);
        outs.push_back((int32_t)v[a].second);
      }
      groups[g].push_back({kv.first, outs});
    }
  }
  const int words = qt + ct + qt * ct;
  std::vector<int32_t> out;
  int nt = 0;
  for (auto& kv : groups) {
    const auto& g = kv.first;
    const auto& lst = kv.second;
    for (size_t s = 0; s < lst.size(); s += ct) {
      std::vector<int32_t> T(words, -1);
      for (int a = 0; a < qt; ++a) T[a] = (int32_t)(a < (int)g.size() ? g[a] : g[0]);
      for (int b = 0; b < ct; ++b) {
        const size_t e = s + b;
        T[qt + b] = (int32_t)(e < lst.size() ? lst[e].first : lst[s].first);
        for (int a = 0; a < qt; ++a)
          T[qt + ct + a * ct + b] =
              (e < lst.size() && a < (int)g.size()) ? lst[e].second[a] : -1;
      }
      out.insert(out.end(), T.begin(), T.end());
      ++nt;
    }
  }
  *n_tiles = nt;
  return out;
}

// Copy host bytes to device memory on `st` through one of the context's
// pinned staging buffers: the first, from the ring position on, whose last
// copy has completed (or, when all are busy, the one at the ring position,
// after its copy completes).
sanns_status stage_upload(sanns_ctx* ctx, void* dst, const void* src, size_t bytes,
                          hipStream_t st) {
  if (!bytes) return SANNS_OK;
  const int K = (int)(sizeof ctx->staging / sizeof ctx->staging[0]);
  int pick = -1;
  for (int i = 0; i < K && pick < 0; ++i) {
    const int j = (ctx->staging_next + i) % K;
    const hipError_t q = hipEventQuery(ctx->staging[j].done);
    if (q == hipSuccess) pick = j;
    else if (q != hipErrorNotReady) return fail(SANNS_E_DEVICE, "staging: %s", hipGetErrorString(q));
  }
  if (pick < 0) {
    pick = ctx->staging_next;
    HIP_TRY(hipEventSynchronize(ctx->staging[pick].done));
  }
  sanns_ctx::Staging& S = ctx->staging[pick];
  ctx->staging_next = (pick + 1) % K;
  if (bytes > S.bytes) {
    // geometric growth: freeing pinned memory waits for the whole device, so
    // a buffer is replaced a handful of times per context, not per size
    const size_t cap = std::max({bytes, 2 * S.bytes, (size_t)1 << 20});
    if (S.buf) HIP_TRY(hipHostFree(S.buf));
    S.buf = nullptr;
    S.bytes = 0;
    HIP_TRY(hipHostMalloc(&S.buf, cap, hipHostMallocDefault));
    S.bytes = cap;
  }
  std::memcpy(S.buf, src, bytes);
  HIP_TRY(hipMemcpyAsync(dst, S.buf, bytes, hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(S.done, st));
  return SANNS_OK;
}

struct WsLayout {
  size_t qntt, tiles, work, tmp, ctrl, qdig, sums, pkntt, flood, total;
};

// mfma: the call runs the matrix-core schedule (query digits and sums regions);
// cp: the circuit-private form (the public keys' NTT form).
WsLayout ws_layout(const sanns_ctx* ctx, uint32_t d, uint32_t Q, uint32_t M, bool mfma,
                   bool cp = false) {
  const size_t N = ctx->p.N, L = ctx->p.L;
  WsLayout w;
  size_t off = 0;
  w.qntt = off;
  off += align256((size_t)Q * d * 2 * L * N * 8);
  w.tiles = off;
  off += align256((size_t)M * 64 * sizeof(int32_t));  // >= M tiles of the largest shape
  w.work = off;
  off += align256((size_t)M * 2 * sizeof(uint32_t));
  w.tmp = off;
  off += align256(2 * L * N * 8);
  w.ctrl = off;  // control words of the persistent schedule
  off += align256(kPersistCtrlWords * sizeof(uint32_t));
  w.qdig = w.sums = off;
  if (mfma) {
    // matrix-core schedule: query digits and slot-major sums (all pairs: C = M / Q)
    off += align256(L * N * 2 * Q * 7 * (size_t)mfma_query_d((int)d));
    w.sums = off;
    off += align256(mfma_sums_bytes((int)Q, (int)((M + Q - 1) / Q), (int)L, ctx->logN));
  }
  w.pkntt = off;
  if (cp) off += align256((size_t)Q * 2 * L * N * 8);
  w.flood = off;  // flood residues [M][L][N] uint64, then e1, e2 [M][2][N] int8
  if (cp) off += align256((size_t)M * L * N * 8 + (size_t)M * 2 * N);
  w.total = off;
  return w;
}

}  // namespace

// ===========================================================================
// context
// ===========================================================================

extern "C" const char* sanns_last_error(void) { return g_last_error.c_str(); }

extern "C" sanns_status sanns_params_derive(uint32_t N, uint32_t L, uint32_t t_bits,
                                           sanns_params* out) {
  if (!out) return fail(SANNS_E_INVALID, "null output");
  if (N < 16 || N > 16384 || (N & (N - 1)))
    return fail(SANNS_E_INVALID, "N = %u is not a power of two in [16, 16384]", N);
  if (L < 1 || L > SANNS_MAX_LIMBS) return fail(SANNS_E_INVALID, "L = %u outside [1, 4]", L);
  if (t_bits < 2 || t_bits > 31) return fail(SANNS_E_INVALID, "t_bits outside [2, 31]");
  std::memset(out, 0, sizeof *out);
  out->N = N;
  out->L = L;
  const auto qs = host::rns_primes(N, L);
  if (qs.size() != L) return fail(SANNS_E_PARAMS, "not enough primes");
  for (uint32_t l = 0; l < L; ++l) out->q[l] = qs[l];
  out->t = host::plain_modulus(N, t_bits);
  out->flags = 0;
  return SANNS_OK;
}

extern "C" sanns_status sanns_ctx_create(const sanns_params* p, int device, sanns_ctx** out) {
  if (!out) return fail(SANNS_E_INVALID, "null output");
  *out = nullptr;
  sanns_status s = check_params(p);
  if (s != SANNS_OK) return s;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev)
    return fail(SANNS_E_INVALID, "device %d outside [0, %d)", device, ndev);
  HIP_TRY(hipSetDevice(device));
  sanns_ctx* ctx = new sanns_ctx();
  ctx->p = *p;
  ctx->device = device;
  ctx->logN = log2u(p->N);
  ctx->digit_db = (p->flags & SANNS_FLAG_DIGIT_DB) != 0;
  const uint32_t N = p->N, L = p->L;
  std::vector<uint64_t> qs(p->q, p->q + L);
  const auto deltas = host::delta_mod_limbs(qs, p->t);
  std::vector<uint64_t> tw_all;
  try {
    for (uint32_t l = 0; l < L; ++l) {
      ctx->ps.p[l] = host::prime_consts(N, qs[l], deltas[l]);
      ctx->ds.c[l] = host::digit_consts(qs[l]);
      const uint64_t psi = host::min_primitive_root_2n(N, qs[l]);
      const auto tw = host::twiddle_table(N, qs[l], psi);
      tw_all.insert(tw_all.end(), tw.begin(), tw.end());
    }
    ctx->dec = host::decode_consts(qs, p->t);
    ctx->flood_bits_max = host::delta_bits(qs, p->t) - 3;
  } catch (const std::exception& e) {
    delete ctx;
    return fail(SANNS_E_PARAMS, "%s", e.what());
  }
  ctx->tone = (uint64_t)((((unsigned __int128)1) << 64) / p->t);
  hipError_t e = hipMalloc(&ctx->d_tw, tw_all.size() * sizeof(uint64_t));
  if (e != hipSuccess) {
    delete ctx;
    return fail(SANNS_E_NOMEM, "twiddle tables: %s", hipGetErrorString(e));
  }
  e = hipMemcpy(ctx->d_tw, tw_all.data(), tw_all.size() * sizeof(uint64_t),
                hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&ctx->d_err, sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(ctx->d_err, 0, sizeof(uint32_t));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
  for (auto& S : ctx->staging) {
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(S.done, ctx->cap_stream);
  }
  if (e != hipSuccess) {
    sanns_ctx_destroy(ctx);
    return fail(SANNS_E_DEVICE, "context setup: %s", hipGetErrorString(e));
  }
  for (uint32_t l = 0; l < L; ++l)
    ctx->tws.tw[l] = reinterpret_cast<const u64x2*>(ctx->d_tw + (size_t)l * 6 * N);
  e = scratch_for_device(device, &ctx->scratch);
  if (e != hipSuccess) {
    sanns_ctx_destroy(ctx);
    return fail(SANNS_E_DEVICE, "scratch address: %s", hipGetErrorString(e));
  }
  *out = ctx;
  return SANNS_OK;
}

extern "C" void sanns_ctx_destroy(sanns_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  for (auto& kv : ctx->graphs) {
    if (kv.second.done) (void)hipEventSynchronize(kv.second.done);
    (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.done) (void)hipEventDestroy(kv.second.done);
  }
  drop_profile_events(ctx);
  for (auto& S : ctx->staging) {
    if (S.done) (void)hipEventSynchronize(S.done);
    if (S.buf) (void)hipHostFree(S.buf);
    if (S.done) (void)hipEventDestroy(S.done);
  }
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->d_tw) (void)hipFree(ctx->d_tw);
  if (ctx->d_err) (void)hipFree(ctx->d_err);
  delete ctx;
}

extern "C" sanns_status sanns_ctx_params(const sanns_ctx* ctx, sanns_params* out) {
  if (!ctx || !out) return fail(SANNS_E_INVALID, "null argument");
  *out = ctx->p;
  return SANNS_OK;
}

extern "C" sanns_status sanns_device_status(sanns_ctx* ctx, void* stream) {
  if (!ctx) return fail(SANNS_E_INVALID, "null context");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  uint32_t v = 0;
  HIP_TRY(hipMemcpy(&v, ctx->d_err, sizeof v, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(ctx->d_err, 0, sizeof v));
  if (v & 1u) return fail(SANNS_E_RANGE, "an input residue was >= its prime");
  if (v & 2u) return fail(SANNS_E_RANGE, "a slot index was outside [-1, n)");
  if (v & 8u) return fail(SANNS_E_RANGE, "a point or norm share was >= t");
  if (v & 4u) return fail(SANNS_E_DEVICE, "the persistent schedule timed out waiting for a phase");
  return SANNS_OK;
}

namespace {
void drop_profile_events(sanns_ctx* ctx) {
  for (auto& call : ctx->prof_events)
    for (auto& e : call) {
      (void)hipEventSynchronize(e.second);
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  ctx->prof_events.clear();
}
}  // namespace

extern "C" sanns_status sanns_profile_enable(sanns_ctx* ctx, int on) {
  if (!ctx) return fail(SANNS_E_INVALID, "null context");
  std::lock_guard<std::mutex> lock(ctx->mu);
  drop_profile_events(ctx);
  ctx->profiling = on != 0;
  return SANNS_OK;
}

extern "C" sanns_status sanns_profile_read(sanns_ctx* ctx, double* ms_out, int* calls) {
  if (!ctx || !ms_out) return fail(SANNS_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lock(ctx->mu);
  double sum[SANNS_N_PHASES] = {};
  for (auto& call : ctx->prof_events)
    for (int p = 0; p < SANNS_N_PHASES; ++p) {
      HIP_TRY(hipEventSynchronize(call[p].second));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, call[p].first, call[p].second));
      sum[p] += ms;
    }
  const int n = (int)ctx->prof_events.size();
  for (int p = 0; p < SANNS_N_PHASES; ++p) ms_out[p] = n ? sum[p] / n : 0.0;
  if (calls) *calls = n;
  return SANNS_OK;
}

extern "C" sanns_status sanns_set_schedule(sanns_ctx* ctx, int lds_variant, int qt, int ct) {
  if (!ctx) return fail(SANNS_E_INVALID, "null context");
  const bool persist = persistent_logn(lds_variant) != 0;
  if (persist && persistent_logn(lds_variant) != ctx->logN)
    return fail(SANNS_E_INVALID, "persistent shape %d is built for N = %d", lds_variant,
                1 << persistent_logn(lds_variant));
  if (lds_variant < 0 || (lds_variant > 0 && !persist && lds_variant != kMfmaSchedule &&
                          mac_lds_min_n(lds_variant) == 0))
    return fail(SANNS_E_INVALID, "LDS variant %d is not built", lds_variant);
  if (lds_variant == kMfmaSchedule && !ctx->digit_db)
    return fail(SANNS_E_INVALID, "schedule %d needs a context with SANNS_FLAG_DIGIT_DB",
                lds_variant);
  if (!(qt == 0 && ct == 0) && mac_tile_bytes(qt, ct) == 0)
    return fail(SANNS_E_INVALID, "tile %dx%d is not built", qt, ct);
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (persist) {
    ctx->force_persist = lds_variant;
  } else {
    ctx->force_lds = lds_variant;
    ctx->force_persist = 0;
  }
  ctx->force_qt = qt;
  ctx->force_ct = ct;
  return SANNS_OK;
}

// ===========================================================================
// database
// ===========================================================================

extern "C" size_t sanns_db_bytes(const sanns_ctx* ctx, uint32_t n_chunks, uint32_t d) {
  if (!ctx) return 0;
  const size_t N = ctx->p.N, L = ctx->p.L;
  size_t b = L * n_chunks * d * N * 8 + (size_t)n_chunks * N * 4;
  if (db_has_digits(ctx, d)) b += mfma_db_bytes((int)n_chunks, (int)d, (int)L, ctx->logN);
  return b;
}

extern "C" sanns_status sanns_encode_db(sanns_ctx* ctx, const void* points, int dtype,
                                        uint64_t n, const int64_t* slot_point,
                                        const sanns_db* db, void* stream) {
  if (!ctx || !points || !slot_point || !db || !db->mem)
    return fail(SANNS_E_INVALID, "null argument");
  if (dtype != SANNS_U8 && dtype != SANNS_I8) return fail(SANNS_E_INVALID, "bad dtype");
  if (db->d == 0 || db->d > SANNS_MAX_D || db->n_chunks == 0 || n == 0)
    return fail(SANNS_E_INVALID, "bad database shape (n=%llu, d=%u, chunks=%u)",
                (unsigned long long)n, db->d, db->n_chunks);
  if (db->bytes < sanns_db_bytes(ctx, db->n_chunks, db->d))
    return fail(SANNS_E_WORKSPACE, "database buffer too small");
  // every squared distance must stay below t (b_d = 2 b_c + ceil(log2 d))
  if ((uint64_t)db->d * 255ull * 255ull >= ctx->p.t)
    return fail(SANNS_E_RANGE, "d * 255^2 = %llu does not fit below t",
                (unsigned long long)db->d * 65025ull);
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const uint32_t N = ctx->p.N, L = ctx->p.L, C = db->n_chunks, d = db->d;
  uint2* res = (uint2*)db->mem;
  uint32_t* norms = (uint32_t*)((char*)db->mem + (size_t)L * C * d * N * 8);
  const uint32_t batch = std::max<uint32_t>(1, std::min<uint32_t>(C, (64u << 20) / (d * N * 2)));
  int16_t* gt = nullptr;
  HIP_TRY(hipMallocAsync((void**)&gt, (size_t)batch * d * N * sizeof(int16_t), st));
  for (uint32_t k0 = 0; k0 < C; k0 += batch) {
    const uint32_t nk = std::min(batch, C - k0);
    HIP_TRY(launch_gather(points, dtype == SANNS_I8, (long)n, (int)d, slot_point,
                          (long)k0 * N, (long)nk * N, ctx->logN, gt, norms, ctx->d_err, st));
    HIP_TRY(launch_encode_ntt(gt, res, (int)k0, (int)nk, (int)C, (int)d, ctx->logN, (int)L,
                              ctx->ps, ctx->tws, st));
  }
  HIP_TRY(hipFreeAsync(gt, st));
  if (db_has_digits(ctx, d)) {
    int8_t* dig = (int8_t*)((char*)db->mem + (size_t)L * C * d * N * 8 + (size_t)C * N * 4);
    HIP_TRY(launch_db_digits(res, dig, (int)C, (int)d, (int)L, ctx->logN, st));
  }
  return SANNS_OK;
}

// ===========================================================================
// client helpers
// ===========================================================================

extern "C" sanns_status sanns_encrypt_query(sanns_ctx* ctx, const int8_t* sk,
                                            const int32_t* msgs, uint32_t Q, uint32_t d,
                                            const uint64_t* a, const int16_t* e,
                                            uint64_t* ct_out, void* stream) {
  if (!ctx || !sk || !msgs || !a || !e || !ct_out) return fail(SANNS_E_INVALID, "null argument");
  if (Q == 0 || d == 0 || d > SANNS_MAX_D) return fail(SANNS_E_INVALID, "bad Q or d");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const uint32_t N = ctx->p.N, L = ctx->p.L;
  uint64_t* sk_ntt = nullptr;
  HIP_TRY(hipMallocAsync((void**)&sk_ntt, (size_t)L * N * 8, st));
  HIP_TRY(launch_sk_ntt(sk, sk_ntt, ctx->logN, (int)L, ctx->ps, ctx->tws, st));
  HIP_TRY(launch_encrypt(a, e, msgs, sk_ntt, ct_out, (int)(Q * d), (int)L, ctx->logN,
                         (uint32_t)ctx->p.t, ctx->ps, ctx->tws, st));
  HIP_TRY(hipFreeAsync(sk_ntt, st));
  return SANNS_OK;
}

extern "C" sanns_status sanns_keygen(sanns_ctx* ctx, uint64_t seed, int8_t* sk, void* stream) {
  if (!ctx || !sk) return fail(SANNS_E_INVALID, "null argument");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(launch_keygen(seed, (int)ctx->p.N, sk, (hipStream_t)stream));
  return SANNS_OK;
}

extern "C" sanns_status sanns_encrypt_query_seeded(sanns_ctx* ctx, const int8_t* sk,
                                                   const int32_t* msgs, uint32_t Q, uint32_t d,
                                                   uint64_t enc_seed, uint64_t* ct_out,
                                                   void* stream) {
  if (!ctx || !sk || !msgs || !ct_out) return fail(SANNS_E_INVALID, "null argument");
  if (Q == 0 || d == 0 || d > SANNS_MAX_D) return fail(SANNS_E_INVALID, "bad Q or d");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const uint32_t N = ctx->p.N, L = ctx->p.L;
  const size_t Qd = (size_t)Q * d;
  uint64_t* a = nullptr;
  int16_t* e = nullptr;
  HIP_TRY(hipMallocAsync((void**)&a, Qd * L * N * 8, st));
  hipError_t err = hipMallocAsync((void**)&e, Qd * N * 2, st);
  if (err == hipSuccess)
    err = launch_sample_enc(enc_seed, 2, 3, (int)Qd, (int)d, (int)L, (int)N, ctx->ps, a, e, st);
  sanns_status s = SANNS_OK;
  if (err == hipSuccess)
    s = sanns_encrypt_query(ctx, sk, msgs, Q, d, a, e, ct_out, stream);
  else
    s = fail(SANNS_E_DEVICE, "seeded encryption: %s", hipGetErrorString(err));
  if (e) (void)hipFreeAsync(e, st);
  (void)hipFreeAsync(a, st);
  return s;
}

extern "C" sanns_status sanns_public_key(sanns_ctx* ctx, const int8_t* sk, uint64_t seed,
                                         uint64_t* pk, void* stream) {
  if (!ctx || !sk || !pk) return fail(SANNS_E_INVALID, "null argument");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const uint32_t N = ctx->p.N, L = ctx->p.L;
  // an encryption of zero whose a and e come from purposes 4 and 5
  char* tmp = nullptr;
  const size_t a_bytes = (size_t)L * N * 8, e_bytes = (size_t)N * 2;
  HIP_TRY(hipMallocAsync((void**)&tmp, a_bytes + e_bytes + 256 + L * N * 8, st));
  uint64_t* a = (uint64_t*)tmp;
  int16_t* e = (int16_t*)(tmp + a_bytes);
  int32_t* zero = (int32_t*)(tmp + a_bytes + e_bytes);
  uint64_t* sk_ntt = (uint64_t*)(tmp + a_bytes + e_bytes + 256);
  hipError_t err = hipMemsetAsync(zero, 0, sizeof(int32_t), st);
  if (err == hipSuccess)
    err = launch_sample_enc(seed, 4, 5, 1, 1, (int)L, (int)N, ctx->ps, a, e, st);
  if (err == hipSuccess) err = launch_sk_ntt(sk, sk_ntt, ctx->logN, (int)L, ctx->ps, ctx->tws, st);
  if (err == hipSuccess)
    err = launch_encrypt(a, e, zero, sk_ntt, pk, 1, (int)L, ctx->logN, (uint32_t)ctx->p.t,
                         ctx->ps, ctx->tws, st);
  (void)hipFreeAsync(tmp, st);
  if (err != hipSuccess) return fail(SANNS_E_DEVICE, "public key: %s", hipGetErrorString(err));
  return SANNS_OK;
}

extern "C" sanns_status sanns_decrypt_shares(sanns_ctx* ctx, const int8_t* sk,
                                             const uint64_t* ct, uint32_t M,
                                             const uint32_t* qnorm2, uint32_t* client_share,
                                             void* stream) {
  if (!ctx || !sk || !ct || !client_share) return fail(SANNS_E_INVALID, "null argument");
  if (M == 0) return SANNS_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const uint32_t N = ctx->p.N, L = ctx->p.L;
  uint64_t* sk_ntt = nullptr;
  HIP_TRY(hipMallocAsync((void**)&sk_ntt, (size_t)L * N * 8, st));
  HIP_TRY(launch_sk_ntt(sk, sk_ntt, ctx->logN, (int)L, ctx->ps, ctx->tws, st));
  HIP_TRY(launch_decrypt(ct, (int)M, sk_ntt, qnorm2, client_share, (int)L, ctx->logN, ctx->ps,
                         ctx->tws, ctx->dec, st));
  HIP_TRY(hipFreeAsync(sk_ntt, st));
  return SANNS_OK;
}

// ===========================================================================
// server hot path
// ===========================================================================

extern "C" size_t sanns_distances_workspace(const sanns_ctx* ctx, const sanns_db* db,
                                            uint32_t Q, uint32_t M, int mode) {
  if (!ctx || !db) return 0;
  const bool mfma = mode != SANNS_MODE_PERSISTENT && mode != SANNS_MODE_PLAIN && Q > 0 &&
                    (uint64_t)M == (uint64_t)Q * db->n_chunks &&
                    call_uses_mfma(ctx, Q, db->n_chunks, db->d, true);
  return ws_layout(ctx, db->d, Q, M, mfma).total;
}

namespace {

// The fused sequence: query NTT, masks, multiply-accumulate, INTT + mask.
// Circuit-private form of a call: the queries' public keys (coefficient form)
// and the workspace for their NTT form, the flood width.
struct CpArgs {
  const uint64_t* pk = nullptr;
  uint64_t* pk_ntt = nullptr;
  uint64_t* flood = nullptr;
  CpConst c{};
  bool on = false;
};

sanns_status enqueue_fused(sanns_ctx* ctx, const sanns_db* db, const uint64_t* ct_in,
                           uint32_t Q, const MaskKey& K, const uint64_t* qids,
                           const uint32_t* dwork, uint32_t M, int qt, int ct, int lds,
                           const void* dtiles, int n_tiles, uint64_t* ct_out,
                           uint32_t* share, uint64_t* qntt, int8_t* qdig, uint64_t* sums,
                           hipStream_t st, bool profile = false, const CpArgs& cp = CpArgs()) {
  const uint32_t N = ctx->p.N, L = ctx->p.L, C = db->n_chunks, d = db->d;
  const bool mfma = lds == kMfmaSchedule;
  const uint2* res = (const uint2*)db->mem;
  const uint32_t* norms = (const uint32_t*)((const char*)db->mem + (size_t)L * C * d * N * 8);
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  if (profile) {
    ev.resize(SANNS_N_PHASES);
    for (auto& e : ev) {
      HIP_TRY(hipEventCreate(&e.first));
      HIP_TRY(hipEventCreate(&e.second));
    }
  }
  auto mark = [&](int phase, bool end) -> hipError_t {
    if (!profile) return hipSuccess;
    return hipEventRecord(end ? ev[phase].second : ev[phase].first, st);
  };
  HIP_TRY(mark(SANNS_PHASE_QUERY_NTT, false));
  HIP_TRY(launch_ntt_fwd(ct_in, qntt, (int)(Q * d * 2 * L), ctx->logN, (int)L, ctx->ps,
                         ctx->tws, ctx->d_err, mfma ? 2 : 1, st, (int)d, (int)(2 * Q)));
  HIP_TRY(mark(SANNS_PHASE_QUERY_NTT, true));
  HIP_TRY(mark(SANNS_PHASE_DIGITS, false));
  if (mfma)
    HIP_TRY(launch_query_digits(qntt, qdig, (int)Q, (int)d, (int)L, ctx->logN, st));
  HIP_TRY(mark(SANNS_PHASE_DIGITS, true));
  HIP_TRY(mark(SANNS_PHASE_MASKS, false));
  if (!mfma)  // the matrix-core schedule draws them in its sums transpose
    HIP_TRY(launch_masks(K, qids, dwork, (int)C, (int)M, ctx->logN, (uint32_t)ctx->p.t,
                         ctx->tone, share, st));
  HIP_TRY(mark(SANNS_PHASE_MASKS, true));
  HIP_TRY(mark(SANNS_PHASE_MAC, false));
  if (mfma) {
    const int8_t* dig = (const int8_t*)db->mem + (size_t)L * C * d * N * 8 + (size_t)C * N * 4;
    HIP_TRY(launch_mac_mfma(qdig, dig, (int)Q, (int)d, (int)C, (int)L, ctx->logN, ctx->ds,
                            sums, st));
  } else if (lds > 0)
    HIP_TRY(launch_mac_lds(lds, (const uint2*)qntt, res, (int)Q, (int)d, (int)L, ctx->logN,
                           (int)C, ctx->ps, ct_out, st));
  else
    HIP_TRY(launch_mac(qt, ct, (const uint2*)qntt, res, dtiles, n_tiles, (int)Q, (int)d, (int)L,
                       ctx->logN, (int)C, ctx->ps, ct_out, st));
  HIP_TRY(mark(SANNS_PHASE_MAC, true));
  HIP_TRY(mark(SANNS_PHASE_SUMS, false));
  if (mfma)
    HIP_TRY(launch_sums_to_ct(sums, ct_out, (int)Q, (int)C, (int)L, ctx->logN, ctx->ps, st, K,
                              qids, (uint32_t)ctx->p.t, ctx->tone, share));
  HIP_TRY(mark(SANNS_PHASE_SUMS, true));
  HIP_TRY(mark(SANNS_PHASE_RERAND, false));
  if (cp.on) {
    HIP_TRY(launch_ntt_fwd(cp.pk, cp.pk_ntt, (int)(Q * 2 * L), ctx->logN, (int)L, ctx->ps,
                           ctx->tws, ctx->d_err, 0, st));
    HIP_TRY(launch_rerand(K, qids, dwork, (int)C, (int)M, (int)L, ctx->logN, cp.pk_ntt, ct_out,
                          ctx->ps, ctx->tws, st));
  }
  HIP_TRY(mark(SANNS_PHASE_RERAND, true));
  HIP_TRY(mark(SANNS_PHASE_INTT_MASK, false));
  if (cp.on)
    HIP_TRY(launch_intt_mask_cp(ct_out, share, norms, dwork, (int)C, (int)M, ctx->logN, (int)L,
                                (uint32_t)ctx->p.t, K, qids, cp.c, ctx->ds, ctx->ps, ctx->tws,
                                cp.flood, st));
  else
    HIP_TRY(launch_intt_mask(ct_out, share, norms, dwork, (int)C, (int)M, ctx->logN, (int)L,
                             (uint32_t)ctx->p.t, ctx->ps, ctx->tws, st));
  HIP_TRY(mark(SANNS_PHASE_INTT_MASK, true));
  if (profile) ctx->prof_events.push_back(ev);
  return SANNS_OK;
}

// One launch per ciphertext operation, in the order a BFV library would issue
// them: NTT(c_i); per chunk: multiply_plain + add over i, INTT, sample mask,
// add_plain.
sanns_status enqueue_plain(sanns_ctx* ctx, const sanns_db* db, const uint64_t* ct_in,
                           uint32_t Q, const MaskKey& K, const uint64_t* qids,
                           const std::vector<uint32_t>& hwork, const uint32_t* dwork,
                           uint32_t M, uint64_t* ct_out, uint32_t* share, uint64_t* qntt,
                           uint64_t* tmp, hipStream_t st) {
  const uint32_t N = ctx->p.N, L = ctx->p.L, C = db->n_chunks, d = db->d;
  const uint2* res = (const uint2*)db->mem;
  const uint32_t* norms = (const uint32_t*)((const char*)db->mem + (size_t)L * C * d * N * 8);
  const size_t ctw = (size_t)2 * L * N;
  for (uint32_t qi = 0; qi < Q; ++qi)
    for (uint32_t i = 0; i < d; ++i)
      HIP_TRY(launch_ntt_fwd(ct_in + ((size_t)qi * d + i) * ctw, qntt + ((size_t)qi * d + i) * ctw,
                             (int)(2 * L), ctx->logN, (int)L, ctx->ps, ctx->tws, ctx->d_err, 1,
                             st));
  for (uint32_t m = 0; m < M; ++m) {
    const uint32_t qi = hwork[2 * m], k = hwork[2 * m + 1];
    uint64_t* acc = ct_out + (size_t)m * ctw;
    for (uint32_t i = 0; i < d; ++i) {
      const uint2* cq = (const uint2*)(qntt + ((size_t)qi * d + i) * ctw);
      if (i == 0) {
        HIP_TRY(launch_mult_plain(cq, res, (int)i, (int)k, (int)d, (int)C, (int)L, ctx->logN,
                                  ctx->ps, acc, st));
      } else {
        HIP_TRY(launch_mult_plain(cq, res, (int)i, (int)k, (int)d, (int)C, (int)L, ctx->logN,
                                  ctx->ps, tmp, st));
        HIP_TRY(launch_add(acc, tmp, (int)L, ctx->logN, ctx->ps, st));
      }
    }
    HIP_TRY(launch_ntt_inv(acc, (int)(2 * L), ctx->logN, (int)L, ctx->ps, ctx->tws, st));
    HIP_TRY(launch_masks(K, qids, dwork + 2 * m, (int)C, 1, ctx->logN, (uint32_t)ctx->p.t,
                         ctx->tone, share + (size_t)m * N, st));
    HIP_TRY(launch_add_plain(acc, share + (size_t)m * N, norms, (int)k, (int)L, ctx->logN,
                             (uint32_t)ctx->p.t, ctx->ps, st));
  }
  return SANNS_OK;
}

}  // namespace

namespace {

// sanns_distances; with noalloc (sanns_distances_noalloc) the call is an
// all-pairs fused launch sequence that allocates nothing: no staging, no
// graph, no profiler events.
sanns_status distances_impl(sanns_ctx* ctx, const sanns_db* db, const uint64_t* ct_in,
                            uint32_t Q, const uint8_t* mask_key, const uint64_t* query_ids,
                            const uint32_t* work, uint32_t M, int mode, uint64_t* ct_out,
                            uint32_t* server_share, void* workspace, size_t ws_bytes,
                            void* stream, bool noalloc, const uint64_t* pk = nullptr,
                            uint32_t flood_bits = 0) {
  if (!ctx || !db || !db->mem || !ct_in || !mask_key || !query_ids || !ct_out ||
      !server_share || !workspace)
    return fail(SANNS_E_INVALID, "null argument");
  if (mode != SANNS_MODE_PLAIN && mode != SANNS_MODE_FUSED && mode != SANNS_MODE_BATCHED &&
      mode != SANNS_MODE_PERSISTENT)
    return fail(SANNS_E_INVALID, "bad mode %d", mode);
  const int pshape = mode == SANNS_MODE_PERSISTENT
                         ? (ctx->force_persist ? ctx->force_persist
                                               : persistent_default_shape(ctx->logN))
                         : 0;
  if (mode == SANNS_MODE_PERSISTENT && pshape == 0)
    return fail(SANNS_E_INVALID, "SANNS_MODE_PERSISTENT needs 2048 <= N <= 16384");
  if (mode == SANNS_MODE_PERSISTENT && db && db->d > (uint32_t)persistent_max_d(pshape))
    return fail(SANNS_E_INVALID, "SANNS_MODE_PERSISTENT needs d <= %d", persistent_max_d(pshape));
  if (Q == 0 || db->d == 0 || db->d > SANNS_MAX_D || db->n_chunks == 0)
    return fail(SANNS_E_INVALID, "bad shape");
  const uint32_t C = db->n_chunks;
  if (!work && (uint64_t)M != (uint64_t)Q * C)
    return fail(SANNS_E_INVALID, "without a work list M must be Q * n_chunks");
  if (M == 0) return SANNS_OK;
  if (work)
    for (uint32_t m = 0; m < M; ++m)
      if (work[2 * m] >= Q || work[2 * m + 1] >= C)
        return fail(SANNS_E_RANGE, "work[%u] = (%u, %u) outside Q x n_chunks", m, work[2 * m],
                    work[2 * m + 1]);
  const bool mfma = mode != SANNS_MODE_PERSISTENT && mode != SANNS_MODE_PLAIN &&
                    call_uses_mfma(ctx, Q, C, db->d, work == nullptr);
  const bool cp_on = pk != nullptr;
  if (cp_on && mode != SANNS_MODE_FUSED && mode != SANNS_MODE_BATCHED)
    return fail(SANNS_E_INVALID, "the circuit-private form runs in SANNS_MODE_FUSED or "
                                 "SANNS_MODE_BATCHED only");
  const WsLayout W = ws_layout(ctx, db->d, Q, M, mfma, cp_on);
  if (ws_bytes < W.total)
    return fail(SANNS_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, W.total);
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  uint64_t* qntt = (uint64_t*)(ws + W.qntt);
  void* dtiles_buf = ws + W.tiles;
  uint32_t* dwork_buf = (uint32_t*)(ws + W.work);
  uint64_t* tmp = (uint64_t*)(ws + W.tmp);
  int8_t* qdig = (int8_t*)(ws + W.qdig);
  uint64_t* sums = (uint64_t*)(ws + W.sums);
  MaskKey K;
  for (int i = 0; i < 8; ++i)
    K.k[i] = (uint32_t)mask_key[4 * i] | (uint32_t)mask_key[4 * i + 1] << 8 |
             (uint32_t)mask_key[4 * i + 2] << 16 | (uint32_t)mask_key[4 * i + 3] << 24;
  CpArgs cp;
  if (cp_on) {
    cp.on = true;
    cp.pk = pk;
    cp.pk_ntt = (uint64_t*)(ws + W.pkntt);
    cp.flood = (uint64_t*)(ws + W.flood);
    cp.c.b = (int)flood_bits;
    for (uint32_t l = 0; l < ctx->p.L; ++l) cp.c.twob[l] = host::pow2_mod((int)flood_bits, ctx->p.q[l]);
  }

  std::lock_guard<std::mutex> lock(ctx->mu);
  if (mode == SANNS_MODE_PLAIN) {
    std::vector<uint32_t> hwork(2 * (size_t)M);
    if (work)
      std::memcpy(hwork.data(), work, hwork.size() * sizeof(uint32_t));
    else
      for (uint32_t m = 0; m < M; ++m) {
        hwork[2 * m] = m / C;
        hwork[2 * m + 1] = m % C;
      }
    sanns_status s = stage_upload(ctx, dwork_buf, hwork.data(), hwork.size() * 4, st);
    if (s != SANNS_OK) return s;
    return enqueue_plain(ctx, db, ct_in, Q, K, query_ids, hwork, dwork_buf, M, ct_out,
                         server_share, qntt, tmp, st);
  }

  int qt, ct, lds;
  double q_per_chunk = Q;
  if (work) {
    std::vector<char> seen(C, 0);
    uint32_t distinct = 0;
    for (uint32_t m = 0; m < M; ++m)
      if (!seen[work[2 * m + 1]]) {
        seen[work[2 * m + 1]] = 1;
        ++distinct;
      }
    q_per_chunk = (double)M / (distinct ? distinct : 1);
  }
  if (ctx->force_lds == kMfmaSchedule && !work && Q >= 2 && !db_has_digits(ctx, db->d))
    return fail(SANNS_E_INVALID,
                "the matrix-core schedule needs SANNS_FLAG_DIGIT_DB, N >= 64 and d <= %d",
                kMfmaMaxD);
  choose_shape(ctx, Q, C, db->d, work == nullptr, q_per_chunk, qt, ct, lds);
  if (pshape) {
    qt = kPersistTileQ;
    ct = kPersistTileC;
    lds = 0;
  }
  const void* dtiles = nullptr;
  const uint32_t* dwork = nullptr;
  int n_tiles;
  if (work) {
    std::vector<int32_t> tiles = build_tiles(work, M, qt, ct, &n_tiles);
    // tiles and the work list go out in one staged copy
    std::vector<char> blob(W.work - W.tiles + (size_t)M * 8);
    std::memcpy(blob.data(), tiles.data(), tiles.size() * 4);
    std::memcpy(blob.data() + (W.work - W.tiles), work, (size_t)M * 8);
    sanns_status s = stage_upload(ctx, dtiles_buf, blob.data(), blob.size(), st);
    if (s != SANNS_OK) return s;
    dtiles = dtiles_buf;
    dwork = dwork_buf;
  } else {
    n_tiles = (int)(((Q + qt - 1) / qt) * ((C + ct - 1) / ct));
  }

  uint32_t* ctrl = (uint32_t*)(ws + W.ctrl);
  auto enqueue = [&](hipStream_t s, bool profile) -> sanns_status {
    if (!pshape)
      return enqueue_fused(ctx, db, ct_in, Q, K, query_ids, dwork, M, qt, ct, lds, dtiles,
                           n_tiles, ct_out, server_share, qntt, qdig, sums, s, profile, cp);
    PersistArgs A;
    A.ct_in = ct_in;
    A.qntt = qntt;
    A.db = (const uint2*)db->mem;
    A.norms = (const uint32_t*)((const char*)db->mem + (size_t)ctx->p.L * C * db->d * ctx->p.N * 8);
    A.qids = query_ids;
    A.work = dwork;
    A.tiles = dtiles;
    A.ct_out = ct_out;
    A.share = server_share;
    A.ctrl = ctrl;
    A.err = ctx->d_err;
    A.Q = (int)Q;
    A.d = (int)db->d;
    A.L = (int)ctx->p.L;
    A.C = (int)C;
    A.M = (int)M;
    A.n_tiles = n_tiles;
    A.t = (uint32_t)ctx->p.t;
    A.tone = ctx->tone;
    A.K = K;
    HIP_TRY(launch_persistent(pshape, A, ctx->ps, ctx->tws, s));
    return SANNS_OK;
  };

  if (noalloc)
    return enqueue_fused(ctx, db, ct_in, Q, K, query_ids, dwork, M, qt, ct, lds, dtiles,
                         n_tiles, ct_out, server_share, qntt, qdig, sums, st, false);
  if (mode == SANNS_MODE_FUSED || (ctx->profiling && !pshape))
    return enqueue_fused(ctx, db, ct_in, Q, K, query_ids, dwork, M, qt, ct, lds, dtiles,
                         n_tiles, ct_out, server_share, qntt, qdig, sums, st, ctx->profiling,
                         cp);

  // batched and persistent: replay (or capture once) the sequence as a hipGraph
  GraphKey key;
  std::memset(&key, 0, sizeof key);
  key.db = db->mem;
  key.C = C;
  key.d = db->d;
  key.Q = Q;
  key.M = M;
  key.ct_in = ct_in;
  key.qids = query_ids;
  key.ct_out = ct_out;
  key.share = server_share;
  key.ws = workspace;
  key.qt = qt;
  key.ct = ct;
  key.lds = lds;
  key.n_tiles = n_tiles;
  key.table = work ? 1 : 0;
  key.persist = pshape;
  key.pk = pk;
  key.flood_bits = flood_bits;
  std::memcpy(key.key, K.k, sizeof K.k);
  auto it = ctx->graphs.find(key);
  if (it == ctx->graphs.end() && ctx->graphs.size() >= kMaxGraphs) {
    // evict the least recently launched graph once its last launch is done
    auto old = ctx->graphs.begin();
    for (auto g = ctx->graphs.begin(); g != ctx->graphs.end(); ++g)
      if (g->second.last_use < old->second.last_use) old = g;
    HIP_TRY(hipEventSynchronize(old->second.done));
    HIP_TRY(hipGraphExecDestroy(old->second.exec));
    HIP_TRY(hipEventDestroy(old->second.done));
    ctx->graphs.erase(old);
  }
  if (it == ctx->graphs.end()) {
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    sanns_status s = enqueue(ctx->cap_stream, false);
    hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (s != SANNS_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    if (e != hipSuccess) return fail(SANNS_E_DEVICE, "capture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(SANNS_E_DEVICE, "instantiate: %s", hipGetErrorString(e));
    sanns_ctx::CachedGraph cg;
    cg.exec = exec;
    e = hipEventCreateWithFlags(&cg.done, hipEventDisableTiming);
    if (e != hipSuccess) {
      (void)hipGraphExecDestroy(exec);
      return fail(SANNS_E_DEVICE, "graph event: %s", hipGetErrorString(e));
    }
    it = ctx->graphs.emplace(key, cg).first;
  }
  HIP_TRY(hipGraphLaunch(it->second.exec, st));
  HIP_TRY(hipEventRecord(it->second.done, st));
  it->second.last_use = ++ctx->graph_clock;
  return SANNS_OK;
}

}  // namespace

extern "C" sanns_status sanns_distances(sanns_ctx* ctx, const sanns_db* db,
                                        const uint64_t* ct_in, uint32_t Q,
                                        const uint8_t* mask_key, const uint64_t* query_ids,
                                        const uint32_t* work, uint32_t M, int mode,
                                        uint64_t* ct_out, uint32_t* server_share,
                                        void* workspace, size_t ws_bytes, void* stream) {
  return distances_impl(ctx, db, ct_in, Q, mask_key, query_ids, work, M, mode, ct_out,
                        server_share, workspace, ws_bytes, stream, false);
}

// ---------------------------------------------------------------------------
// gathered chunks: per-call chunks of retrieved points (or of secret shares)
// ---------------------------------------------------------------------------

namespace {

// Chunks encoded per gather/encode round (their 32-bit plaintexts stay below
// 64 MiB).
uint32_t gather_batch(uint32_t d, uint32_t N, uint32_t M) {
  return std::max<uint32_t>(1, std::min<uint32_t>(M, (64u << 20) / (d * N * 4)));
}

struct GatherLayout {
  size_t db, gt, inner, total, db_bytes;
};

// Ct: chunks of the resident tail database appended to the call's chunks.
GatherLayout gather_layout(const sanns_ctx* ctx, uint32_t d, uint32_t Q, uint32_t M,
                           uint32_t Ct) {
  const size_t N = ctx->p.N, L = ctx->p.L, C = (size_t)M + Ct;
  GatherLayout g;
  g.db = 0;
  g.db_bytes = L * C * d * N * 8 + C * N * 4;  // residues, then norms
  g.gt = align256(g.db_bytes);
  g.inner = g.gt + align256((size_t)gather_batch(d, (uint32_t)N, M) * d * N * 4);
  g.total = g.inner + ws_layout(ctx, d, Q, M + Q * Ct, false).total;
  return g;
}

}  // namespace

extern "C" sanns_status sanns_slot_ranges(const int64_t* start, const int64_t* len,
                                          const int64_t* off, uint32_t R, int64_t* slot_point,
                                          uint64_t total, void* stream) {
  if (!slot_point || (R && (!start || !len || !off))) return fail(SANNS_E_INVALID, "null argument");
  if (total > (1ull << 40)) return fail(SANNS_E_INVALID, "total too large");
  HIP_TRY(launch_slot_ranges(start, len, off, (int)R, slot_point, (long)total, (hipStream_t)stream));
  return SANNS_OK;
}

extern "C" size_t sanns_distances_gathered_workspace(const sanns_ctx* ctx, uint32_t d, uint32_t Q,
                                                     uint32_t M, const sanns_db* tail) {
  if (!ctx || d == 0 || M == 0) return 0;
  return gather_layout(ctx, d, Q, M, tail ? tail->n_chunks : 0).total;
}

extern "C" sanns_status sanns_distances_gathered(
    sanns_ctx* ctx, const void* points, int dtype, uint64_t n, uint32_t d,
    const uint32_t* norm_shares, const int64_t* slot_point, const uint32_t* row_query,
    uint32_t M, const sanns_db* tail, const uint64_t* ct_in, uint32_t Q,
    const uint8_t* mask_key, const uint64_t* query_ids, uint64_t* ct_out,
    uint32_t* server_share, void* workspace, size_t ws_bytes, void* stream) {
  if (!ctx || !points || !slot_point || !row_query || !ct_in || !mask_key || !query_ids ||
      !ct_out || !server_share || !workspace)
    return fail(SANNS_E_INVALID, "null argument");
  if (tail && (!tail->mem || tail->d != d || tail->n_chunks == 0))
    return fail(SANNS_E_INVALID, "the tail database must have dimension d and chunks");
  if (dtype != SANNS_U8 && dtype != SANNS_I8 && dtype != SANNS_SHARE32)
    return fail(SANNS_E_INVALID, "bad dtype");
  if (dtype == SANNS_SHARE32 && !norm_shares)
    return fail(SANNS_E_INVALID, "SANNS_SHARE32 needs the norm shares");
  if (n == 0 || d == 0 || d > SANNS_MAX_D || Q == 0 || M == 0)
    return fail(SANNS_E_INVALID, "bad shape (n=%llu, d=%u, Q=%u, M=%u)", (unsigned long long)n,
                d, Q, M);
  if (dtype != SANNS_SHARE32 && (uint64_t)d * 255ull * 255ull >= ctx->p.t)
    return fail(SANNS_E_RANGE, "d * 255^2 = %llu does not fit below t",
                (unsigned long long)d * 65025ull);
  for (uint32_t m = 0; m < M; ++m)
    if (row_query[m] >= Q)
      return fail(SANNS_E_RANGE, "row_query[%u] = %u outside [0, Q)", m, row_query[m]);
  const uint32_t Ct = tail ? tail->n_chunks : 0, C = M + Ct;
  const uint64_t rows = (uint64_t)M + (uint64_t)Q * Ct;
  if (rows > 0x7FFFFFFFull) return fail(SANNS_E_INVALID, "too many output rows");
  const GatherLayout G = gather_layout(ctx, d, Q, M, Ct);
  if (ws_bytes < G.total)
    return fail(SANNS_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, G.total);
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const uint32_t N = ctx->p.N, L = ctx->p.L;
  char* ws = (char*)workspace;
  uint2* res = (uint2*)(ws + G.db);
  uint32_t* norms = (uint32_t*)(ws + G.db + (size_t)L * C * d * N * 8);
  int32_t* gt = (int32_t*)(ws + G.gt);
  const uint32_t batch = gather_batch(d, N, M);
  const int kind = dtype == SANNS_SHARE32 ? 2 : (dtype == SANNS_I8 ? 1 : 0);
  for (uint32_t k0 = 0; k0 < M; k0 += batch) {
    const uint32_t nk = std::min(batch, M - k0);
    HIP_TRY(launch_gather32(points, kind, (long)n, (int)d, norm_shares, (uint32_t)ctx->p.t,
                            slot_point, (long)k0 * N, (long)nk * N, ctx->logN, gt, norms,
                            ctx->d_err, st));
    HIP_TRY(launch_encode_ntt32(gt, res, (int)k0, (int)nk, (int)C, (int)d, ctx->logN, (int)L,
                                ctx->ps, ctx->tws, st));
  }
  if (Ct) {
    // the tail's resident NTT form and norms follow the gathered chunks
    const size_t plane = (size_t)d * N;  // uint2 words of one chunk and limb
    const uint2* tres = (const uint2*)tail->mem;
    for (uint32_t l = 0; l < L; ++l)
      HIP_TRY(hipMemcpyAsync(res + ((size_t)l * C + M) * plane, tres + (size_t)l * Ct * plane,
                             (size_t)Ct * plane * sizeof(uint2), hipMemcpyDeviceToDevice, st));
    const uint32_t* tnorms = (const uint32_t*)((const char*)tail->mem + (size_t)L * Ct * plane * 8);
    HIP_TRY(hipMemcpyAsync(norms + (size_t)M * N, tnorms, (size_t)Ct * N * 4,
                           hipMemcpyDeviceToDevice, st));
  }
  sanns_db tmp;
  tmp.mem = res;
  tmp.bytes = G.db_bytes;
  tmp.n_chunks = C;
  tmp.d = d;
  std::vector<uint32_t> work(2 * (size_t)rows);
  for (uint32_t m = 0; m < M; ++m) {
    work[2 * m] = row_query[m];
    work[2 * m + 1] = m;
  }
  for (uint32_t q = 0; q < Q; ++q)
    for (uint32_t k = 0; k < Ct; ++k) {
      const size_t r = (size_t)M + (size_t)q * Ct + k;
      work[2 * r] = q;
      work[2 * r + 1] = M + k;
    }
  return distances_impl(ctx, &tmp, ct_in, Q, mask_key, query_ids, work.data(), (uint32_t)rows,
                        SANNS_MODE_FUSED, ct_out, server_share, ws + G.inner, G.total - G.inner,
                        stream, false);
}

// ---------------------------------------------------------------------------
// k-means of the balanced clustering
// ---------------------------------------------------------------------------

extern "C" size_t sanns_kmeans_workspace(uint32_t k, uint32_t d) {
  if (k == 0 || d == 0 || d > 256) return 0;
  return km_workspace((int)k, (int)d);
}

namespace {
sanns_status km_check(const int8_t* points, uint64_t n, uint32_t d, uint32_t k, size_t ws_bytes,
                      const void* ws) {
  if (!points || !ws) return fail(SANNS_E_INVALID, "null argument");
  if (n == 0 || d == 0 || d > 256 || k == 0 || n >= (1ull << 40) || k >= (1u << 30))
    return fail(SANNS_E_INVALID, "bad shape (n=%llu, d=%u, k=%u)", (unsigned long long)n, d, k);
  if (ws_bytes < km_workspace((int)k, (int)d))
    return fail(SANNS_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes,
                km_workspace((int)k, (int)d));
  return SANNS_OK;
}
}  // namespace

extern "C" sanns_status sanns_kmeans_init(const int8_t* points, uint64_t n, uint32_t d,
                                          const int64_t* idx, uint32_t k, int32_t* centers,
                                          uint32_t* bad, void* stream) {
  if (!points || !idx || !centers || !bad) return fail(SANNS_E_INVALID, "null argument");
  if (n == 0 || d == 0 || d > 256 || k == 0) return fail(SANNS_E_INVALID, "bad shape");
  HIP_TRY(launch_km_init(points, (long)n, (int)d, idx, (int)k, centers, bad, (hipStream_t)stream));
  return SANNS_OK;
}

extern "C" sanns_status sanns_kmeans_assign(const int8_t* points, uint64_t n, uint32_t d,
                                            const int32_t* centers, uint32_t k,
                                            const int32_t* prev, int32_t* assign,
                                            uint32_t* changed, void* workspace,
                                            size_t ws_bytes, void* stream) {
  sanns_status s = km_check(points, n, d, k, ws_bytes, workspace);
  if (s != SANNS_OK) return s;
  if (!centers || !assign) return fail(SANNS_E_INVALID, "null argument");
  HIP_TRY(launch_km_assign(points, (long)n, (int)d, centers, (int)k, prev, assign, changed,
                           workspace, (hipStream_t)stream));
  return SANNS_OK;
}

extern "C" sanns_status sanns_kmeans_update(const int8_t* points, uint64_t n, uint32_t d,
                                            const int32_t* assign, uint32_t k, int32_t* centers,
                                            int64_t* counts, void* workspace, size_t ws_bytes,
                                            void* stream) {
  sanns_status s = km_check(points, n, d, k, ws_bytes, workspace);
  if (s != SANNS_OK) return s;
  if (!centers || !assign) return fail(SANNS_E_INVALID, "null argument");
  HIP_TRY(launch_km_update(points, (long)n, (int)d, assign, (int)k, centers, counts, workspace,
                           (hipStream_t)stream));
  return SANNS_OK;
}

extern "C" uint32_t sanns_flood_bits(const sanns_ctx* ctx) {
  return ctx ? (uint32_t)ctx->flood_bits_max : 0u;
}

extern "C" size_t sanns_distances_cp_workspace(const sanns_ctx* ctx, const sanns_db* db,
                                               uint32_t Q, uint32_t M, int mode) {
  if (!ctx || !db) return 0;
  const bool mfma = mode != SANNS_MODE_PERSISTENT && mode != SANNS_MODE_PLAIN && Q > 0 &&
                    (uint64_t)M == (uint64_t)Q * db->n_chunks &&
                    call_uses_mfma(ctx, Q, db->n_chunks, db->d, true);
  return ws_layout(ctx, db->d, Q, M, mfma, true).total;
}

extern "C" sanns_status sanns_distances_cp(sanns_ctx* ctx, const sanns_db* db,
                                           const uint64_t* ct_in, uint32_t Q,
                                           const uint8_t* mask_key, const uint64_t* query_ids,
                                           const uint64_t* pk, uint32_t flood_bits,
                                           const uint32_t* work, uint32_t M, int mode,
                                           uint64_t* ct_out, uint32_t* server_share,
                                           void* workspace, size_t ws_bytes, void* stream) {
  if (!ctx || !pk) return fail(SANNS_E_INVALID, "null argument");
  if (flood_bits == 0) flood_bits = (uint32_t)ctx->flood_bits_max;
  if ((int)flood_bits > ctx->flood_bits_max)
    return fail(SANNS_E_RANGE, "flood_bits %u exceeds %d (2^b must stay within Delta / 4)",
                flood_bits, ctx->flood_bits_max);
  return distances_impl(ctx, db, ct_in, Q, mask_key, query_ids, work, M, mode, ct_out,
                        server_share, workspace, ws_bytes, stream, false, pk, flood_bits);
}

extern "C" sanns_status sanns_distances_noalloc(sanns_ctx* ctx, const sanns_db* db,
                                                const uint64_t* ct_in, uint32_t Q,
                                                const uint8_t* mask_key,
                                                const uint64_t* query_ids, uint64_t* ct_out,
                                                uint32_t* server_share, void* stream) {
  if (!ctx || !db) return fail(SANNS_E_INVALID, "null argument");
  if (!ctx->scratch) return fail(SANNS_E_DEVICE, "no scratch address for device %d", ctx->device);
  const uint64_t M = (uint64_t)Q * db->n_chunks;
  if (M > 0xFFFFFFFFull) return fail(SANNS_E_INVALID, "Q * n_chunks overflows");
  const size_t need = sanns_distances_workspace(ctx, db, Q, (uint32_t)M, SANNS_MODE_FUSED);
  if (need > (size_t)SANNS_NOALLOC_SCRATCH_BYTES)
    return fail(SANNS_E_WORKSPACE,
                "the call needs %zu bytes of scratch, more than the %u bytes the library holds "
                "per device (SANNS_NOALLOC_SCRATCH_BYTES); use sanns_distances with a workspace",
                need, (unsigned)SANNS_NOALLOC_SCRATCH_BYTES);
  return distances_impl(ctx, db, ct_in, Q, mask_key, query_ids, nullptr, (uint32_t)M,
                        SANNS_MODE_FUSED, ct_out, server_share, ctx->scratch,
                        (size_t)SANNS_NOALLOC_SCRATCH_BYTES, stream, true);
}
