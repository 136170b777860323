// C ABI of libepi3 (declared in include/epi3.h): argument checks, buffer
// carving and kernel sequencing.  All arithmetic of the scan runs in the
// kernels; the host computes sizes, the class split of the samples and the
// log-factorial tables.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "epi3_internal.h"

using namespace epi3;

namespace {

constexpr int64_t kAlign = 256;

struct Carver {
  char *base;
  int64_t off = 0;
  explicit Carver(void *b) : base(static_cast<char *>(b)) {}
  template <typename T>
  T *take(int64_t n) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += n * (int64_t)sizeof(T);
    return p;
  }
  int64_t size() const { return (off + kAlign - 1) / kAlign * kAlign; }
};

int32_t snp_stride(int32_t M) { return (M + kSnpPad - 1) / kSnpPad * kSnpPad + kSnpPad; }
int32_t words_of(int64_t n) { return (int32_t)((n + 31) / 32); }
int32_t byte_stride(int32_t N) { return (N + 255) / 256 * 256; }

struct EncodeLayout {
  int32_t Mp, W0, W1, Wtot, classes, S;
  uint32_t *planes;
  uint8_t *bytes;
  uint8_t *nibbles;
  int32_t *pairs;
  double *lf64;
  float *lf32;
  int32_t *list;
  int32_t *status;
  int64_t total;
};

EncodeLayout encode_layout(void *buf, int32_t M, int32_t n1, int32_t n0, int32_t layout) {
  EncodeLayout L{};
  const int32_t N = n0 + n1;
  L.Mp = snp_stride(M);
  if (layout == EPI3_LAYOUT_SPLIT) {
    L.W0 = words_of(n0);
    L.W1 = words_of(n1);
    L.Wtot = L.W0 + L.W1;
    L.classes = 2;
    L.S = byte_stride(n0 > n1 ? n0 : n1);
  } else {
    L.W0 = L.W1 = words_of(N);
    L.Wtot = L.W0;
    L.classes = 1;
    L.S = byte_stride(N);
  }
  Carver c(buf);
  L.status = c.take<int32_t>(64);
  L.planes = c.take<uint32_t>((int64_t)L.Wtot * L.Mp * 2);
  L.bytes = c.take<uint8_t>((int64_t)L.classes * L.Mp * 2 * L.S);
  L.nibbles = c.take<uint8_t>((int64_t)L.classes * L.Mp * 2 * (L.S / 2));
  L.pairs = c.take<int32_t>((int64_t)L.classes * L.Mp * L.Mp * 4);
  L.lf64 = c.take<double>((int64_t)N + 2);
  L.lf32 = c.take<float>((int64_t)N + 2);
  L.list = c.take<int32_t>((int64_t)L.Wtot * 32);
  L.total = c.size();
  return L;
}

// Log factorials L[n] = sum_{b=1}^{n} log b, summed in increasing b (the
// inner sums of Eq. 1), n = 0..nmax.
void host_log_factorials(int64_t nmax, std::vector<double> &L64, std::vector<float> &L32) {
  L64.assign(nmax + 1, 0.0);
  L32.assign(nmax + 1, 0.f);
  double acc = 0.0;
  for (int64_t n = 1; n <= nmax; ++n) {
    acc = acc + log((double)n);
    L64[n] = acc;
  }
  for (int64_t n = 0; n <= nmax; ++n) L32[n] = (float)L64[n];
}

// The tables are sequential sums, so the table up to a smaller n is a prefix
// of a longer one: the process keeps the longest built so far and encodes
// copy their prefix (building 16k entries costs about 0.14 ms of host time
// per call otherwise).  Superseded tables stay alive until the process ends,
// so a copy still reading one is never left without its source.
struct LfTables {
  std::vector<double> L64;
  std::vector<float> L32;
};
static const LfTables *log_factorial_tables(int64_t nmax) {
  static std::mutex m;
  static std::vector<LfTables *> built;
  std::lock_guard<std::mutex> g(m);
  if (built.empty() || (int64_t)built.back()->L64.size() < nmax + 1) {
    LfTables *t = new LfTables;
    host_log_factorials(nmax, t->L64, t->L32);
    built.push_back(t);
  }
  return built.back();
}

double log_factorial_at(int64_t n) {
  double acc = 0.0;
  for (int64_t b = 1; b <= n; ++b) acc = acc + log((double)b);
  return acc;
}

// Workspace of one plain scan.
struct ScanLayout {
  Job *job;
  int64_t *jprefix;
  unsigned long long *queue;
  SelJob *sel;
  SelState *st;
  uint32_t *hist;
  float *score;
  int64_t *cand;
  uint32_t *candkey;
  CandRec *rec;
  uint64_t *skey;         // sort buffers (candidate capacities above kRankDirectMax)
  uint32_t *sidx;
  epi3_hit *hits;
  uint32_t *ckey;         // compacted low end of the plane
  int64_t *crank;
  int64_t ccap;
  PlainJob *pjob;         // matrix-core variants: the job record
  int64_t *jbegin;        // and its tile range [2]
  uint8_t *scratch;       // matrix-core variants: two buffers of pass_tiles tiles
  int64_t pass_tiles;
  int64_t cap;
  // bounded selection (no score plane; matrix-core variants): every
  // sample_stride-th tile is scored first into a sample plane, whose k-th
  // smallest score bounds what the full pass appends to the list ckey / crank
  bool bounded;
  int64_t sample_stride, sample_tiles;
  float *sample;          // [sample_tiles][4096]
  SelJob *ssel;           // selection of the k-th sample score
  SelState *sst;
  uint32_t *shist;
  int64_t total;
};

int64_t default_cap(int64_t T, int32_t k, int64_t cand_cap) {
  int64_t cap = cand_cap > 0 ? cand_cap : std::max<int64_t>(4096, 4 * (int64_t)k);
  if (T > 0 && cap > T) cap = T;
  return std::max<int64_t>(cap, 1);
}

constexpr int64_t kPlainPassBytes = 1ll << 30;  // per scratch buffer of the plain matrix-core path

// Tile rules registered by epi3_tile_rule (process-wide).
struct TileRule {
  int32_t variant, min_snps, min_samples, tile;
};
struct Tiles {
  std::mutex mu;
  std::vector<TileRule> rules;
  int64_t pass_bytes = 0;
  int64_t compact_cap = 0;
  int32_t batch_select = EPI3_BATCH_SELECT_AUTO;
  int32_t scan_select = EPI3_SCAN_SELECT_AUTO;
  uint64_t gen = 0;  // bumped by every setter: part of the cached graphs' key
};
Tiles &tiles() {
  static Tiles t;
  return t;
}
// The applicable rule's tile for (variant, M, N), or `dflt`.
int rule_tile(int32_t variant, int32_t M, int32_t N, int dflt) {
  Tiles &t = tiles();
  std::lock_guard<std::mutex> g(t.mu);
  const TileRule *best = nullptr;
  for (const TileRule &r : t.rules) {
    if (r.variant != variant || r.min_snps > M || r.min_samples > N) continue;
    if (!best || r.min_snps > best->min_snps ||
        (r.min_snps == best->min_snps && r.min_samples >= best->min_samples))
      best = &r;
  }
  return best ? best->tile : dflt;
}
int batch_select_mode() {
  Tiles &t = tiles();
  std::lock_guard<std::mutex> g(t.mu);
  return t.batch_select;
}
// Phenotype batches of at least this many triplets select by bound (AUTO).
constexpr int64_t kBoundedMinTriplets = 1ll << 22;

int scan_select_mode() {
  Tiles &t = tiles();
  std::lock_guard<std::mutex> g(t.mu);
  return t.scan_select;
}
// Plain scans whose FP32 score plane would exceed this many bytes select by
// bound (AUTO): beyond about 2900 SNPs.
constexpr int64_t kPlainPlaneMaxBytes = 16ll << 30;

uint64_t settings_gen() {
  Tiles &t = tiles();
  std::lock_guard<std::mutex> g(t.mu);
  return t.gen;
}
int64_t pass_bytes(int64_t dflt) {
  Tiles &t = tiles();
  std::lock_guard<std::mutex> g(t.mu);
  return t.pass_bytes > 0 ? t.pass_bytes : dflt;
}

int64_t compact_cap_override() {
  Tiles &t = tiles();
  std::lock_guard<std::mutex> g(t.mu);
  return t.compact_cap;
}

// Capacity of the compacted low end of a score plane of T triplets.
int64_t compact_cap(int64_t T, int64_t cap) {
  int64_t c = 16 * cap > 65536 ? 16 * cap : 65536;
  {
    Tiles &t = tiles();
    std::lock_guard<std::mutex> g(t.mu);
    if (t.compact_cap > 0) c = t.compact_cap;
  }
  return c < T ? c : (T > 0 ? T : 1);
}

// The matrix-core count kernels address the value planes with 32-bit byte
// offsets, and the plain finish kernel the two classes' pair tables with
// 32-bit entry indices.
bool offsets32_ok(const epi3_dataset &d) {
  const int64_t classes = d.layout == EPI3_LAYOUT_SPLIT ? 2 : 1;
  const int64_t value_bytes = classes * d.snp_stride * 2 * (int64_t)d.byte_stride;
  const int64_t pair_entries = classes * d.snp_stride * (int64_t)d.snp_stride;
  return value_bytes <= 0xffffffffll && pair_entries <= 0xffffffffll;
}

bool mfma_supported(const epi3_dataset &d) {
  return d.bytes && d.nibbles && d.n_cases <= 65535 && d.n_controls <= 65535 && offsets32_ok(d);
}

// Count-kernel choice for a SPLIT data set (a variant, or a negative status).
int plain_variant(const epi3_dataset &d, int32_t variant) {
  if (variant < EPI3_VARIANT_AUTO || variant > EPI3_VARIANT_MFMA_FP4) return EPI3_E_INVALID;
  if (variant == EPI3_VARIANT_AUTO) {
    const int v = rule_tile(EPI3_VARIANT_AUTO, d.n_snps, d.n_samples, EPI3_VARIANT_VALU);
    return v != EPI3_VARIANT_VALU && mfma_supported(d) ? v : EPI3_VARIANT_VALU;
  }
  if (variant != EPI3_VARIANT_VALU && !mfma_supported(d)) return EPI3_E_UNSUPPORTED;
  return variant;
}

int pick_JB(const epi3_dataset &d, int32_t v) { return rule_tile(v, d.n_snps, d.n_samples, 4); }

ScanLayout scan_layout(void *ws, const epi3_dataset &d, int32_t k, int64_t cand_cap,
                       int32_t variant) {
  ScanLayout L{};
  const int64_t T = epi3_n_triplets(d.n_snps);
  L.cap = default_cap(T, k, cand_cap);
  Carver c(ws);
  L.job = c.take<Job>(1);
  L.jprefix = c.take<int64_t>((int64_t)d.n_snps + 1);
  L.queue = c.take<unsigned long long>(4);
  L.sel = c.take<SelJob>(1);
  L.st = c.take<SelState>(1);
  L.hist = c.take<uint32_t>(kHistBins);
  const int smode = scan_select_mode();
  // (AUTO: only data sets the matrix cores can count; a vector-ALU scan of a
  // larger one needs EPI3_SCAN_SELECT_PLANE)
  L.bounded = T > 0 && (smode == EPI3_SCAN_SELECT_BOUNDED ||
                        (smode == EPI3_SCAN_SELECT_AUTO && 4 * T > kPlainPlaneMaxBytes &&
                         mfma_supported(d)));
  // (epi3_topk reads the state and the hits: their places depend on k,
  // cand_cap and the selection mode only, not on the variant)
  if (!L.bounded) L.score = c.take<float>(T);
  L.cand = c.take<int64_t>(L.cap);
  L.candkey = c.take<uint32_t>(L.cap);
  L.rec = c.take<CandRec>(L.cap);
  L.skey = c.take<uint64_t>(sort_len(L.cap));
  L.sidx = c.take<uint32_t>(sort_len(L.cap));
  L.hits = c.take<epi3_hit>(std::max<int32_t>(k, 1));
  const int v = plain_variant(d, variant);
  const bool mfma = v == EPI3_VARIANT_MFMA || v == EPI3_VARIANT_MFMA_FP4;
  const int JB = mfma ? pick_JB(d, v) : 0;
  if (L.bounded && mfma) {
    // about max(1024, 8 k) sample tiles (4096 scores each) spread evenly over
    // the tile order, enough of them to hold k triplets
    const int64_t tiles = host_plain_tiles(d.n_snps, JB);
    const int64_t want = std::max<int64_t>(1024, 8 * (int64_t)k);
    int64_t stride = std::max<int64_t>(1, tiles / want), ns = 0;
    while (stride > 1 && host_plain_sample_valid(d.n_snps, JB, stride, &ns) < k) stride /= 2;
    host_plain_sample_valid(d.n_snps, JB, stride, &ns);
    L.sample_stride = stride;
    L.sample_tiles = ns;
    L.sample = c.take<float>(ns * 4096);
    L.ssel = c.take<SelJob>(1);
    L.sst = c.take<SelState>(1);
    L.shist = c.take<uint32_t>(kHistBins);
  }
  L.ccap = compact_cap(T, L.cap);
  if (L.bounded && mfma && compact_cap_override() <= 0) {
    // the list: twice the expected count (the sample holds one tile in
    // sample_stride, so about k sample_stride scores lie below its k-th),
    // plus slack; a size set by epi3_set_compact_cap is taken as it is
    L.ccap = std::max(L.ccap, std::min<int64_t>(T, 2 * (int64_t)k * L.sample_stride + 65536));
  }
  L.ckey = c.take<uint32_t>(L.ccap);
  L.crank = c.take<int64_t>(L.ccap);
  L.pjob = c.take<PlainJob>(1);
  L.jbegin = c.take<int64_t>(2);
  if (T > 0 && mfma) {
    const int64_t tiles = host_plain_tiles(d.n_snps, JB);
    L.pass_tiles = std::max<int64_t>(
        1, std::min<int64_t>(tiles, pass_bytes(kPlainPassBytes) / kPlainTileScratch));
    L.scratch = c.take<uint8_t>(2 * L.pass_tiles * kPlainTileScratch);
  }
  L.total = c.size();
  return L;
}

// Workspace of one scan of another interaction order (2: pairs, 4: quads).
struct OrderLayout {
  SelJob *sel;
  SelState *st;
  uint32_t *hist;
  float *score;
  int64_t *cand;
  uint32_t *candkey;
  CandRec *rec;
  uint64_t *skey;
  uint32_t *sidx;
  uint8_t *hits;
  uint32_t *ckey;
  int64_t *crank;
  int64_t ccap;
  int64_t cap;
  uint8_t *t3;  // quads: triplet corner table (NULL: counted per quad)
  // quads on the matrix cores (data sets with FP4 value planes)
  bool qmfma;
  int64_t *qprefix;           // [M + 1] tiles before each pivot j
  unsigned long long *queue;  // tile queue
  uint8_t *qscratch;          // pass_tiles tiles of corner cells
  int64_t pass_tiles;
  int64_t total;
};

constexpr int32_t kQuadMaxSnps = 4096;
constexpr int64_t kQuadPassBytes = 2ll << 30;  // per corner scratch buffer of the matrix-core quad scan

int64_t order_combos(int order, int32_t M) { return order == 2 ? c2(M) : c4(M); }
int64_t order_hit_bytes(int order) {
  return order == 2 ? (int64_t)sizeof(epi3_pair_hit) : (int64_t)sizeof(epi3_quad_hit);
}

OrderLayout order_layout(void *ws, const epi3_dataset &d, int order, int32_t k, int64_t cand_cap) {
  OrderLayout L{};
  const int64_t T = order_combos(order, d.n_snps);
  L.cap = default_cap(T, k, cand_cap);
  Carver c(ws);
  L.sel = c.take<SelJob>(1);
  L.st = c.take<SelState>(1);
  L.hist = c.take<uint32_t>(kHistBins);
  L.score = c.take<float>(T);
  L.cand = c.take<int64_t>(L.cap);
  L.candkey = c.take<uint32_t>(L.cap);
  L.rec = c.take<CandRec>(L.cap);
  L.skey = c.take<uint64_t>(sort_len(L.cap));
  L.sidx = c.take<uint32_t>(sort_len(L.cap));
  L.hits = c.take<uint8_t>(std::max<int32_t>(k, 1) * order_hit_bytes(order));
  L.ccap = compact_cap(T, L.cap);
  L.ckey = c.take<uint32_t>(L.ccap);
  L.crank = c.take<int64_t>(L.ccap);
  if (order == 4 && d.n_cases <= 65535 && d.n_controls <= 65535)
    L.t3 = c.take<uint8_t>(quad_triplet_table_bytes(d.n_snps));
  if (order == 4 && T > 0 && mfma_supported(d)) {
    L.qmfma = true;
    L.qprefix = c.take<int64_t>((int64_t)d.n_snps + 1);
    L.queue = c.take<unsigned long long>(4);
    const int64_t tiles = host_quad_tiles(d.n_snps);
    L.pass_tiles = std::max<int64_t>(
        1, std::min<int64_t>(tiles, pass_bytes(kQuadPassBytes) / kQuadTileScratch));
    L.qscratch = c.take<uint8_t>(2 * L.pass_tiles * kQuadTileScratch);  // two buffers
  }
  L.total = c.size();
  return L;
}

bool valid_dataset(const epi3_dataset *d) {
  return d && d->n_snps >= 0 && d->n_samples > 0 && d->planes && d->pairs && d->lf64 && d->lf32 &&
         d->status && (d->layout == EPI3_LAYOUT_SPLIT || d->layout == EPI3_LAYOUT_MASKED);
}

#define HIP_OK(expr)                        \
  do {                                      \
    if ((expr) != hipSuccess) return EPI3_E_HIP; \
  } while (0)

Job make_job(const epi3_dataset &d, float *score, uint32_t *counts, int64_t *jprefix,
             uint32_t *keyrange, int P) {
  Job J{};
  J.planes = static_cast<const uint32_t *>(d.planes);
  J.pairs = d.pairs;
  J.score = score;
  J.jprefix = jprefix;
  J.counts = counts;
  J.keyrange = keyrange;
  J.tile_begin = 0;
  J.n_tiles = host_tiles(d.n_snps, P);
  J.T = epi3_n_triplets(d.n_snps);
  J.M = d.n_snps;
  J.Mp = d.snp_stride;
  J.W0 = d.words[0];
  J.W1 = d.words[1];
  J.N0 = d.n_controls;
  J.N1 = d.n_cases;
  J.P = P;
  return J;
}

SelJob make_seljob(const epi3_dataset &d, const float *score, int64_t T, SelState *st,
                   uint32_t *hist, int64_t *cand, uint32_t *candkey, CandRec *rec, epi3_hit *hits,
                   int64_t cap, int32_t k, uint32_t *ckey, int64_t *crank, int64_t ccap) {
  SelJob S{};
  S.candkey = candkey;
  S.ckey = ckey;
  S.crank = crank;
  S.ccap = ccap;
  S.score = score;
  S.T = T;
  S.st = st;
  S.hist = hist;
  S.cand = cand;
  S.rec = rec;
  S.hits = hits;
  S.cap = cap;
  S.err2 = 2.0 * epi3_k2_error_bound(d.n_samples);
  S.planes = static_cast<const uint32_t *>(d.planes);
  S.pairs = d.pairs;
  S.case_pairs = nullptr;
  S.case_mask = nullptr;
  S.n1_dev = nullptr;
  S.case_stride = 1;
  S.lf64 = d.lf64;
  S.M = d.n_snps;
  S.Mp = d.snp_stride;
  S.W0 = d.words[0];
  S.W1 = d.words[1];
  S.N0 = d.n_controls;
  S.N1 = d.n_cases;
  S.layout = d.layout;
  S.k = k;
  S.sample = sample_select(T, k) ? 1 : 0;
  return S;
}

int pick_P(const epi3_dataset &d) {
  return rule_tile(EPI3_VARIANT_VALU, d.n_snps, d.n_samples, tile_P_default(d.n_snps, d.n_samples));
}

// Second stream and events of the count / finish overlap of one matrix-core
// scan.  A call holds a context of its own (AuxLease) for as long as it
// enqueues work and hands it back before it returns, so two calls running at
// the same time never record or wait on the same events, and a graph capture
// forks only its own context's stream.  A context handed back may still have
// the previous call's finish kernels queued on its stream: the next holder's
// work queues behind them (an ordering, never a mix of data: every wait is
// issued while its event's latest record is the holder's own).
struct AuxCtx {
  hipStream_t s2 = nullptr;
  hipEvent_t ev[5] = {};
};
struct AuxPool {
  std::mutex mu;
  std::vector<AuxCtx *> idle;
};
AuxPool &aux_pool() {
  static AuxPool p;
  return p;
}
void aux_destroy(AuxCtx *c) {
  for (hipEvent_t e : c->ev)
    if (e) (void)hipEventDestroy(e);
  if (c->s2) (void)hipStreamDestroy(c->s2);
  delete c;
}
AuxCtx *aux_make(int *rc) {
  AuxCtx *c = new AuxCtx;
  *rc = EPI3_OK;
  if (hipStreamCreateWithFlags(&c->s2, hipStreamNonBlocking) != hipSuccess) *rc = EPI3_E_HIP;
  for (int x = 0; x < 5 && *rc == EPI3_OK; ++x)
    if (hipEventCreateWithFlags(&c->ev[x], hipEventDisableTiming) != hipSuccess) *rc = EPI3_E_HIP;
  if (*rc != EPI3_OK) {
    aux_destroy(c);
    return nullptr;
  }
  return c;
}
struct AuxLease {
  AuxCtx *c = nullptr;
  int rc = EPI3_OK;
  AuxLease() {
    AuxPool &p = aux_pool();
    {
      std::lock_guard<std::mutex> g(p.mu);
      if (!p.idle.empty()) {
        c = p.idle.back();
        p.idle.pop_back();
        return;
      }
    }
    c = aux_make(&rc);
  }
  ~AuxLease() {
    if (!c) return;
    AuxPool &p = aux_pool();
    std::lock_guard<std::mutex> g(p.mu);
    p.idle.push_back(c);
  }
  AuxLease(const AuxLease &) = delete;
  AuxLease &operator=(const AuxLease &) = delete;
};

// ---- optional kernel timing: HIP events on the call's stream ----
struct Timing {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> rec[5];  // 0: count, 1: selection, 2: batched, 3: finish, 4: pairwise tables
};
Timing &timing() {
  static Timing t;
  return t;
}

hipEvent_t take_event() {
  Timing &t = timing();
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records an event pair around `fn` when timing is on.
template <typename F>
int timed(int which, hipStream_t s, F &&fn) {
  Timing &t = timing();
  hipEvent_t a = nullptr, b = nullptr;
  {
    std::lock_guard<std::mutex> g(t.mu);
    if (t.on) {
      a = take_event();
      b = take_event();
    }
  }
  if (a && b && hipEventRecord(a, s) != hipSuccess) return EPI3_E_HIP;
  const int rc = fn();
  if (a && b) {
    if (hipEventRecord(b, s) != hipSuccess) return EPI3_E_HIP;
    std::lock_guard<std::mutex> g(t.mu);
    t.rec[which].push_back({a, b});
  }
  return rc;
}

// Buffers of a matrix-core plain count over one or more data sets: two
// scratch buffers of pass_tiles tiles, the jobs' PlainJob records and their
// first global tiles, and the tile queue.
struct MfmaBufs {
  uint8_t *scratch;
  int64_t pass_tiles;
  PlainJob *pjobs;            // [n]
  int64_t *job_begin;         // [n + 1]
  unsigned long long *queue;
};

// One data set of a matrix-core plain count.
struct MfmaTask {
  const epi3_dataset *d;
  float *score;
  uint32_t *counts;           // optional tables [T][2][27]
  int64_t *jprefix;           // [M + 1]
  uint32_t *keyrange;         // [2]
};

// Bounded selection of a single-task matrix-core count (see ScanLayout).
struct PlainBound {
  int64_t stride, sample_tiles;
  float *sample;
  SelJob *ssel, *sel;  // device: selection of the sample's k-th score, the main selection
  SelState *sst, *st;
  uint32_t *ckey;
  int64_t *crank;
  int64_t ccap;
};

// Counts and scores every triplet of the tasks' data sets (all with the same
// operand type and tile JB) in one sequence of passes over their tiles taken
// in task order: data set x owns global tiles job_begin[x] .. job_begin[x + 1]
// and the persistent count and finish kernels walk the global tile order, so
// one data set's last tiles share a launch with the next one's first.  With
// `bd` (one task): a sample pass over every bd->stride-th tile first, its k-th
// smallest score + 2 e(N) as the bound, then the full pass appending only the
// scores under the bound to the list (no score plane).
int enqueue_count_mfma(const std::vector<MfmaTask> &tasks, bool fp4, int JB, const MfmaBufs &W,
                       hipStream_t s, AuxCtx *ctx, const PlainBound *bd = nullptr) {
  if (bd && tasks.size() != 1) return EPI3_E_INVALID;
  const int32_t unit = fp4 ? 128 : 64;  // samples per 64-byte staged chunk
  const int n = (int)tasks.size();
  std::vector<int64_t> begin(n + 1, 0);
  const float *lf32 = nullptr;
  int32_t lf_len = 0;
  for (int x = 0; x < n; ++x) {
    const epi3_dataset &d = *tasks[x].d;
    PlainJob pj{};
    pj.vals = static_cast<const uint8_t *>(fp4 ? d.nibbles : d.bytes);
    pj.pairs = d.pairs;
    pj.score = tasks[x].score;
    pj.counts = tasks[x].counts;
    pj.keyrange = tasks[x].keyrange;
    pj.jprefix = tasks[x].jprefix;
    pj.n_tiles = host_plain_tiles(d.n_snps, JB);
    pj.T = epi3_n_triplets(d.n_snps);
    pj.M = d.n_snps;
    pj.Mp = d.snp_stride;
    pj.Sb = fp4 ? d.byte_stride / 2 : d.byte_stride;
    pj.Sb0 = (d.n_controls + unit - 1) / unit * 64;
    pj.Sb1 = (d.n_cases + unit - 1) / unit * 64;
    pj.N0 = d.n_controls;
    pj.N1 = d.n_cases;
    pj.JB = JB;
    if (pj.Sb0 > pj.Sb || pj.Sb1 > pj.Sb) return EPI3_E_INVALID;
    HIP_OK(launch_write_plainjob(pj, W.pjobs + x, s));
    HIP_OK(launch_plain_prefix(W.pjobs + x, s));
    begin[x + 1] = begin[x] + pj.n_tiles;
    // log factorials are prefix sums, so the longest table serves every set
    if (d.n_samples + 2 > lf_len) {
      lf_len = d.n_samples + 2;
      lf32 = d.lf32;
    }
  }
  const int64_t tiles = begin[n];
  if (tiles == 0) return EPI3_OK;
  HIP_OK(launch_write_i64(begin.data(), n + 1, W.job_begin, s));
  const bool counts = n > 0 && tasks[0].counts != nullptr;
  uint4 *buf[2] = {reinterpret_cast<uint4 *>(W.scratch),
                   reinterpret_cast<uint4 *>(W.scratch + W.pass_tiles * kPlainTileScratch)};
  // Pass p counts into scratch buffer p % 2 on `s`; its finish kernel runs on
  // the second stream while `s` counts pass p + 1.  Count p + 2 waits for
  // finish p (same buffer).  The slots of a pass are the tiles n0 + q of a
  // sequence of n_all tiles 0, stride, 2 stride, ...
  hipStream_t s2 = ctx->s2;
  hipEvent_t ev_start = ctx->ev[0], ev_cnt[2] = {ctx->ev[1], ctx->ev[2]},
             ev_fin[2] = {ctx->ev[3], ctx->ev[4]};
  auto passes = [&](int64_t n_all, int64_t stride, PlainOut out) -> int {
    HIP_OK(hipEventRecord(ev_start, s));
    HIP_OK(hipStreamWaitEvent(s2, ev_start, 0));
    int p = 0;
    for (int64_t n0 = 0; n0 < n_all; n0 += W.pass_tiles, ++p) {
      const int64_t nn = std::min(W.pass_tiles, n_all - n0);
      const int b = p & 1;
      if (p >= 2) HIP_OK(hipStreamWaitEvent(s, ev_fin[b], 0));
      HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(W.queue), 0u, 2, s));
      int rc = timed(0, s, [&]() {
        return launch_count_mfma_plain(W.pjobs, W.job_begin, n, JB, fp4, buf[b], n0 * stride, nn,
                                       stride, W.queue, s) == hipSuccess
                   ? EPI3_OK
                   : EPI3_E_HIP;
      });
      if (rc != EPI3_OK) return rc;
      HIP_OK(hipEventRecord(ev_cnt[b], s));
      HIP_OK(hipStreamWaitEvent(s2, ev_cnt[b], 0));
      out.stride = stride;
      out.sample_base = n0;
      rc = timed(3, s2, [&]() {
        return launch_finish_plain(W.pjobs, W.job_begin, n, JB, buf[b], n0 * stride, nn, lf32,
                                   lf_len, counts, out, s2) == hipSuccess
                   ? EPI3_OK
                   : EPI3_E_HIP;
      });
      if (rc != EPI3_OK) return rc;
      HIP_OK(hipEventRecord(ev_fin[b], s2));
    }
    HIP_OK(hipEventRecord(ev_fin[0], s2));
    HIP_OK(hipStreamWaitEvent(s, ev_fin[0], 0));
    return EPI3_OK;
  };
  PlainOut out{};
  if (!bd) {
    out.mode = kPermOutPlane;
    return passes(tiles, 1, out);
  }
  if (counts) return EPI3_E_INVALID;
  // sample pass: slots of no triplet stay +inf
  HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(bd->sample), 0x7f800000u,
                         bd->sample_tiles * 4096, s));
  out.mode = kPermOutSample;
  out.sample = bd->sample;
  out.range = &bd->sst->kmin;
  int rc = passes(bd->sample_tiles, bd->stride, out);
  if (rc != EPI3_OK) return rc;
  HIP_OK(launch_select_kth(bd->ssel, 1, bd->sample_tiles * 4096, s));
  HIP_OK(launch_sample_bound(bd->sel, bd->ssel, 1, s));
  PlainOut bo{};
  bo.mode = kPermOutBounded;
  bo.st = bd->st;
  bo.ckey = bd->ckey;
  bo.crank = bd->crank;
  bo.ccap = bd->ccap;
  return passes(tiles, 1, bo);
}

}  // namespace

// Scans of another interaction order (2: pairs, 4: quads) on a SPLIT data set.
static int order_check(const epi3_dataset *d, int order, int32_t k) {
  if (!valid_dataset(d) || k <= 0) return EPI3_E_INVALID;
  if (d->layout != EPI3_LAYOUT_SPLIT) return EPI3_E_UNSUPPORTED;
  if (order == 4 && d->n_snps > kQuadMaxSnps) return EPI3_E_UNSUPPORTED;
  return EPI3_OK;
}

static int64_t order_workspace_bytes(const epi3_dataset *d, int order, int32_t k, int64_t cand_cap) {
  const int rc = order_check(d, order, k);
  if (rc != EPI3_OK) return rc;
  return order_layout(nullptr, *d, order, k, cand_cap).total;
}

static double order_error_bound(int order, int32_t n_samples);

static int order_scan(const epi3_dataset *d, int order, int32_t k, int64_t cand_cap, void *ws_dev,
               int64_t ws_bytes, void *stream) {
  int rc = order_check(d, order, k);
  if (rc != EPI3_OK) return rc;
  if (!ws_dev || reinterpret_cast<uintptr_t>(ws_dev) % kAlign) return EPI3_E_INVALID;
  OrderLayout W = order_layout(ws_dev, *d, order, k, cand_cap);
  if (ws_bytes < W.total) return EPI3_E_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t T = order_combos(order, d->n_snps);
  SelJob S = make_seljob(*d, W.score, T, W.st, W.hist, W.cand, W.candkey, W.rec, nullptr, W.cap, k,
                         W.ckey, W.crank, W.ccap);
  S.order = order;
  S.skey = W.skey;
  S.sidx = W.sidx;
  S.sortP = sort_len(W.cap);
  if (order == 2) S.pair_hits = reinterpret_cast<epi3_pair_hit *>(W.hits);
  else S.quad_hits = reinterpret_cast<epi3_quad_hit *>(W.hits);
  S.err2 = 2.0 * order_error_bound(order, d->n_samples);
  HIP_OK(launch_write_seljobs(&S, 1, W.sel, s));
  HIP_OK(launch_init_select(W.sel, 1, s));
  if (T > 0 && W.qmfma) {
    // quads on the matrix cores: pass p of tiles is counted (timed as the
    // count stage) into scratch buffer p % 2 on `s`; its finish kernel (timed
    // as table completion) runs on the library's second stream while `s`
    // counts pass p + 1, and count p + 2 waits for finish p (same buffer)
    HIP_OK(launch_triplet_corners(*d, W.t3, s));
    HIP_OK(launch_quad_prefix(d->n_snps, W.qprefix, s));
    AuxLease lease;
    if (lease.rc != EPI3_OK) return lease.rc;
    hipStream_t s2 = lease.c->s2;
    hipEvent_t ev_start = lease.c->ev[0], ev_cnt[2] = {lease.c->ev[1], lease.c->ev[2]},
               ev_fin[2] = {lease.c->ev[3], lease.c->ev[4]};
    uint8_t *buf[2] = {W.qscratch, W.qscratch + W.pass_tiles * kQuadTileScratch};
    HIP_OK(hipEventRecord(ev_start, s));
    HIP_OK(hipStreamWaitEvent(s2, ev_start, 0));
    const int64_t tiles = host_quad_tiles(d->n_snps);
    int p = 0;
    for (int64_t t0 = 0; t0 < tiles; t0 += W.pass_tiles, ++p) {
      const int64_t nn = std::min(W.pass_tiles, tiles - t0);
      const int b = p & 1;
      if (p >= 2) HIP_OK(hipStreamWaitEvent(s, ev_fin[b], 0));
      HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(W.queue), 0u, 2, s));
      rc = timed(0, s, [&]() {
        return launch_count_mfma_quad(*d, W.qprefix, W.queue, t0, nn, buf[b], s) == hipSuccess
                   ? EPI3_OK
                   : EPI3_E_HIP;
      });
      if (rc != EPI3_OK) return rc;
      HIP_OK(hipEventRecord(ev_cnt[b], s));
      HIP_OK(hipStreamWaitEvent(s2, ev_cnt[b], 0));
      rc = timed(3, s2, [&]() {
        return launch_finish_quad(*d, buf[b], W.qprefix, W.t3, t0, nn, W.score, &W.st->kmin,
                                  s2) == hipSuccess
                   ? EPI3_OK
                   : EPI3_E_HIP;
      });
      if (rc != EPI3_OK) return rc;
      HIP_OK(hipEventRecord(ev_fin[b], s2));
    }
    // everything back on `s` before the selection reads the plane
    HIP_OK(hipEventRecord(ev_fin[0], s2));
    HIP_OK(hipStreamWaitEvent(s, ev_fin[0], 0));
  } else if (T > 0) {
    rc = timed(0, s, [&]() {
      const hipError_t e = order == 2 ? launch_pair_scores(*d, W.score, &W.st->kmin, s)
                                      : launch_quad_scores(*d, W.t3, W.score, &W.st->kmin, s);
      return e == hipSuccess ? EPI3_OK : EPI3_E_HIP;
    });
    if (rc != EPI3_OK) return rc;
  }
  return timed(1, s, [&]() {
    return launch_select(W.sel, 1, T, W.cap, k, S.sample != 0, s) == hipSuccess ? EPI3_OK
                                                                                : EPI3_E_HIP;
  });
}

static int order_topk(const epi3_dataset *d, int order, int32_t k, int64_t cand_cap, void *ws_dev,
               void *hits_host, int32_t *n_out, void *stream) {
  const int rc = order_check(d, order, k);
  if (rc != EPI3_OK) return rc;
  if (!ws_dev || !hits_host || !n_out) return EPI3_E_INVALID;
  OrderLayout W = order_layout(ws_dev, *d, order, k, cand_cap);
  hipStream_t s = static_cast<hipStream_t>(stream);
  SelState st;
  int32_t status = 0;
  HIP_OK(hipMemcpyAsync(&st, W.st, sizeof(st), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(&status, d->status, sizeof(status), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  *n_out = 0;
  if (status & 1) return EPI3_E_GENOTYPE;
  if ((int64_t)st.ncand > W.cap) {
    *n_out = (int32_t)std::min<unsigned long long>(st.ncand, 0x7fffffffull);
    return EPI3_E_CAPACITY;
  }
  const int64_t keff = st.keff;
  if (keff > 0) {
    HIP_OK(hipMemcpyAsync(hits_host, W.hits, keff * order_hit_bytes(order), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
  }
  *n_out = (int32_t)keff;
  return EPI3_OK;
}

static int order_score_plane(const epi3_dataset *d, int order, int32_t k, int64_t cand_cap, void *ws_dev,
                      float **plane_dev) {
  const int rc = order_check(d, order, k);
  if (rc != EPI3_OK) return rc;
  if (!ws_dev || !plane_dev) return EPI3_E_INVALID;
  *plane_dev = order_layout(ws_dev, *d, order, k, cand_cap).score;
  return EPI3_OK;
}

extern "C" {

const char *epi3_version(void) { return "epi3 0.1 (gfx950)"; }

int64_t epi3_n_triplets(int32_t n_snps) { return c3(n_snps); }

double epi3_k2_error_bound(int32_t n_samples) {
  // Per row the FP32 evaluation of L[r+1] - (L[r0] + L[r1]) with table entries
  // rounded to FP32 errs by at most 4u L[r+1] (u = 2^-24; L is superadditive so
  // L[r0] + L[r1] <= L[r+1]); summing 27 rows adds at most 26u sum_rows L[r+1];
  // and sum_rows L[r+1] <= L[N + 27].  32u L[N + 27] covers both plus the
  // second-order terms and the FP64 evaluation's own rounding.
  if (n_samples < 0) return 0.0;
  return 32.0 * ldexp(1.0, -24) * log_factorial_at((int64_t)n_samples + 27);
}

double epi3_k2_error_bound_pairs(int32_t n_samples) {
  // As for triplets with 9 rows: 4u L[r+1] per row, 8u sum_rows L[r+1] for
  // the summation, sum_rows L[r+1] <= L[N + 9]; 14u L[N + 9] covers both plus
  // the second-order terms and the FP64 evaluation's own rounding.
  if (n_samples < 0) return 0.0;
  return 14.0 * ldexp(1.0, -24) * log_factorial_at((int64_t)n_samples + 9);
}

int64_t epi3_n_pairs(int32_t n_snps) { return c2(n_snps); }

double epi3_k2_error_bound_quads(int32_t n_samples) {
  // As for triplets with 81 rows: 4u L[r+1] per row, 80u sum_rows L[r+1] for
  // the summation, sum_rows L[r+1] <= L[N + 81]; 86u L[N + 81] covers both plus
  // the second-order terms and the FP64 evaluation's own rounding.
  if (n_samples < 0) return 0.0;
  return 86.0 * ldexp(1.0, -24) * log_factorial_at((int64_t)n_samples + 81);
}

int64_t epi3_n_quads(int32_t n_snps) { return c4(n_snps); }

int64_t epi3_encode_bytes(int32_t n_snps, int32_t n_cases, int32_t n_controls, int32_t layout) {
  if (n_snps < 0 || n_cases < 0 || n_controls < 0 || n_cases + n_controls <= 0) return EPI3_E_INVALID;
  if (layout == (EPI3_LAYOUT_SPLIT | EPI3_ENCODE_BITS_ONLY)) layout = EPI3_LAYOUT_SPLIT;
  if (layout != EPI3_LAYOUT_SPLIT && layout != EPI3_LAYOUT_MASKED) return EPI3_E_INVALID;
  return encode_layout(nullptr, n_snps, n_cases, n_controls, layout).total;
}

int epi3_encode(const uint8_t *geno_dev, int64_t ld, const uint8_t *pheno_host, int32_t n_snps,
                int32_t n_samples, int32_t layout, void *buf_dev, int64_t buf_bytes, void *stream,
                epi3_dataset *out) {
  if (!out || !pheno_host || !buf_dev || n_snps < 0 || n_samples <= 0 || ld < n_samples ||
      (n_snps > 0 && !geno_dev))
    return EPI3_E_INVALID;
  const bool values = layout != (EPI3_LAYOUT_SPLIT | EPI3_ENCODE_BITS_ONLY);
  if (!values) layout = EPI3_LAYOUT_SPLIT;
  if (layout != EPI3_LAYOUT_SPLIT && layout != EPI3_LAYOUT_MASKED) return EPI3_E_INVALID;
  if (reinterpret_cast<uintptr_t>(buf_dev) % kAlign) return EPI3_E_INVALID;
  int32_t n1 = 0;
  for (int32_t s = 0; s < n_samples; ++s) {
    if (pheno_host[s] > 1) return EPI3_E_PHENOTYPE;
    n1 += pheno_host[s];
  }
  const int32_t n0 = n_samples - n1;
  EncodeLayout L = encode_layout(buf_dev, n_snps, n1, n0, layout);
  if (buf_bytes < L.total) return EPI3_E_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);

  // sample list per output word: controls then cases (SPLIT), or all (MASKED)
  std::vector<int32_t> list((size_t)L.Wtot * 32, -1);
  if (layout == EPI3_LAYOUT_SPLIT) {
    int32_t p0 = 0, p1 = L.W0 * 32;
    for (int32_t x = 0; x < n_samples; ++x) {
      if (pheno_host[x]) list[p1++] = x; else list[p0++] = x;
    }
  } else {
    for (int32_t x = 0; x < n_samples; ++x) list[x] = x;
  }
  const LfTables *lt = log_factorial_tables((int64_t)n_samples + 1);
  const size_t n_lf = (size_t)n_samples + 2;  // L[0 .. n_samples + 1]

  HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(L.status), 0u, 64, s));
  HIP_OK(hipMemcpyAsync(L.list, list.data(), list.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(L.lf64, lt->L64.data(), n_lf * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(L.lf32, lt->L32.data(), n_lf * sizeof(float), hipMemcpyHostToDevice, s));
  HIP_OK(launch_encode(geno_dev, ld, L.list, n_snps, L.Mp, layout == EPI3_LAYOUT_SPLIT ? L.W0 : L.Wtot,
                       layout == EPI3_LAYOUT_SPLIT ? L.W1 : 0, L.planes, L.status, s));
  if (layout == EPI3_LAYOUT_MASKED)
    HIP_OK(launch_encode_values(geno_dev, ld, L.list, 0, n_samples, 0, 0, 1, n_snps, L.Mp, L.S,
                                L.bytes, L.nibbles, s));
  else if (values)
    HIP_OK(launch_encode_values(geno_dev, ld, L.list, 0, n0, L.W0 * 32, n1, 2, n_snps, L.Mp, L.S,
                                L.bytes, L.nibbles, s));
  const int prc = timed(4, s, [&]() {
    return launch_pairs(L.planes, L.Mp, n_snps, L.W0, layout == EPI3_LAYOUT_SPLIT ? L.W1 : 0,
                        L.classes, nullptr, L.pairs, s) == hipSuccess
               ? EPI3_OK
               : EPI3_E_HIP;
  });
  if (prc != EPI3_OK) return prc;
  HIP_OK(hipStreamSynchronize(s));  // host vectors above must outlive the copies

  memset(out, 0, sizeof(*out));
  out->n_snps = n_snps;
  out->n_samples = n_samples;
  out->n_cases = n1;
  out->n_controls = n0;
  out->words[0] = L.W0;
  out->words[1] = L.W1;
  out->layout = layout;
  out->snp_stride = L.Mp;
  out->byte_stride = L.S;
  out->planes = L.planes;
  out->bytes = values ? L.bytes : nullptr;
  out->nibbles = values ? L.nibbles : nullptr;
  out->pairs = L.pairs;
  out->lf64 = L.lf64;
  out->lf32 = L.lf32;
  out->status = L.status;
  return EPI3_OK;
}

int64_t epi3_workspace_bytes(const epi3_dataset *d, int32_t k, int32_t variant, int64_t cand_cap) {
  if (!valid_dataset(d) || k <= 0) return EPI3_E_INVALID;
  const int v = plain_variant(*d, variant);
  if (v < 0) return v;
  return scan_layout(nullptr, *d, k, cand_cap, variant).total;
}

// bounded: select by bound (W.bounded; matrix-core variants only) instead of
// scoring into `score`
static int enqueue_count(const epi3_dataset &d, int32_t variant, float *score, uint32_t *counts,
                         const ScanLayout &W, hipStream_t s, bool bounded = false) {
  const int v = plain_variant(d, variant);
  if (v < 0) return v;
  if (v == EPI3_VARIANT_MFMA || v == EPI3_VARIANT_MFMA_FP4) {
    if (!W.scratch) return EPI3_E_WORKSPACE;
    const MfmaBufs B{W.scratch, W.pass_tiles, W.pjob, W.jbegin, W.queue};
    AuxLease lease;
    if (lease.rc != EPI3_OK) return lease.rc;
    const std::vector<MfmaTask> one{{&d, score, counts, W.jprefix, &W.st->kmin}};
    if (bounded) {
      const PlainBound bd{W.sample_stride, W.sample_tiles, W.sample, W.ssel, W.sel,
                          W.sst,           W.st,           W.ckey,   W.crank, W.ccap};
      return enqueue_count_mfma(one, v == EPI3_VARIANT_MFMA_FP4, pick_JB(d, v), B, s, lease.c,
                                &bd);
    }
    return enqueue_count_mfma(one, v == EPI3_VARIANT_MFMA_FP4, pick_JB(d, v), B, s, lease.c);
  }
  if (bounded) return EPI3_E_UNSUPPORTED;
  const int P = pick_P(d);
  Job J = make_job(d, score, counts, W.jprefix, &W.st->kmin, P);
  HIP_OK(launch_write_jobs(&J, 1, W.job, s));
  HIP_OK(launch_tile_prefix(W.job, 1, s));
  HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(W.queue), 0u, 2, s));
  return timed(0, s, [&]() {
    return launch_count_valu(W.job, 1, J.n_tiles, W.queue, d.lf32, d.n_samples + 2, P, P,
                             counts != nullptr, s) == hipSuccess
               ? EPI3_OK
               : EPI3_E_HIP;
  });
}

int epi3_scan(const epi3_dataset *d, int32_t k, int32_t variant, int64_t cand_cap, void *ws_dev,
              int64_t ws_bytes, void *stream) {
  if (!valid_dataset(d) || k <= 0 || !ws_dev) return EPI3_E_INVALID;
  if (d->layout != EPI3_LAYOUT_SPLIT) return EPI3_E_INVALID;
  if (reinterpret_cast<uintptr_t>(ws_dev) % kAlign) return EPI3_E_INVALID;
  const int v = plain_variant(*d, variant);
  if (v < 0) return v;
  ScanLayout W = scan_layout(ws_dev, *d, k, cand_cap, variant);
  if (W.bounded && !W.sample) return EPI3_E_UNSUPPORTED;  // the vector-ALU count writes a plane
  if (ws_bytes < W.total) return EPI3_E_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t T = epi3_n_triplets(d->n_snps);
  SelJob S = make_seljob(*d, W.score, T, W.st, W.hist, W.cand, W.candkey, W.rec, W.hits, W.cap, k,
                         W.ckey, W.crank, W.ccap);
  S.skey = W.skey;
  S.sidx = W.sidx;
  S.sortP = sort_len(W.cap);
  if (W.bounded) S.sample = 1;  // the list is built before the selection starts
  HIP_OK(launch_write_seljobs(&S, 1, W.sel, s));
  HIP_OK(launch_init_select(W.sel, 1, s));
  if (W.bounded) {
    // selection of the k-th smallest sample score (the sample plane read whole)
    SelJob ss = make_seljob(*d, W.sample, W.sample_tiles * 4096, W.sst, W.shist, nullptr, nullptr,
                            nullptr, nullptr, 1, k, nullptr, nullptr, 0);
    ss.sample = 0;
    HIP_OK(launch_write_seljobs(&ss, 1, W.ssel, s));
    HIP_OK(launch_init_select(W.ssel, 1, s));
  }
  if (T > 0) {
    const int rc = enqueue_count(*d, variant, W.score, nullptr, W, s, W.bounded);
    if (rc != EPI3_OK) return rc;
  }
  // a bounded scan's selection reads its list only: size the grids for that;
  // its sample flag only says that the list exists (the selection's sample
  // phase reads a score plane, so it runs for plane jobs only)
  const int64_t sel_T = W.bounded ? W.ccap : T;
  const bool sampled = S.sample != 0 && S.score != nullptr;
  return timed(1, s, [&]() {
    return launch_select(W.sel, 1, sel_T, W.cap, k, sampled, s) == hipSuccess ? EPI3_OK
                                                                              : EPI3_E_HIP;
  });
}

int epi3_topk(const epi3_dataset *d, int32_t k, int64_t cand_cap, void *ws_dev, epi3_hit *hits_host,
              int32_t *n_out, void *stream) {
  if (!valid_dataset(d) || k <= 0 || !ws_dev || !hits_host || !n_out) return EPI3_E_INVALID;
  ScanLayout W = scan_layout(ws_dev, *d, k, cand_cap, EPI3_VARIANT_VALU);
  hipStream_t s = static_cast<hipStream_t>(stream);
  SelState st;
  int32_t status = 0;
  HIP_OK(hipMemcpyAsync(&st, W.st, sizeof(st), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(&status, d->status, sizeof(status), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  *n_out = 0;
  if (status & 1) return EPI3_E_GENOTYPE;
  if (st.done == 3u) {
    // the bounded list overflowed: 16 x cand_cap entries hold it on a retry
    const int64_t need = std::max<int64_t>((int64_t)((st.cn + 15) / 16), W.cap + 1);
    *n_out = (int32_t)std::min<int64_t>(need, 0x7fffffff);
    return EPI3_E_CAPACITY;
  }
  if ((int64_t)st.ncand > W.cap) {
    *n_out = (int32_t)std::min<unsigned long long>(st.ncand, 0x7fffffffull);
    return EPI3_E_CAPACITY;
  }
  const int64_t keff = st.keff;
  if (keff > 0) {
    HIP_OK(hipMemcpyAsync(hits_host, W.hits, keff * sizeof(epi3_hit), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
  }
  *n_out = (int32_t)keff;
  return EPI3_OK;
}

int epi3_score_plane(const epi3_dataset *d, int32_t k, int64_t cand_cap, void *ws_dev,
                     float **plane_dev) {
  if (!valid_dataset(d) || k <= 0 || !ws_dev || !plane_dev) return EPI3_E_INVALID;
  const ScanLayout W = scan_layout(ws_dev, *d, k, cand_cap, EPI3_VARIANT_VALU);
  if (W.bounded) return EPI3_E_UNSUPPORTED;
  *plane_dev = W.score;
  return EPI3_OK;
}

int epi3_scan_tables(const epi3_dataset *d, int32_t variant, uint32_t *counts_dev, float *k2_dev,
                     void *ws_dev, int64_t ws_bytes, void *stream) {
  if (!valid_dataset(d) || !k2_dev || !ws_dev) return EPI3_E_INVALID;
  if (d->layout != EPI3_LAYOUT_SPLIT) return EPI3_E_INVALID;
  const int v = plain_variant(*d, variant);
  if (v < 0) return v;
  ScanLayout W = scan_layout(ws_dev, *d, 1, 0, variant);
  if (ws_bytes < W.total) return EPI3_E_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t T = epi3_n_triplets(d->n_snps);
  if (T == 0) return EPI3_OK;
  HIP_OK(launch_fill_u32(&W.st->kmin, 0xffffffffu, 1, s));
  HIP_OK(launch_fill_u32(&W.st->kmax, 0u, 1, s));
  return enqueue_count(*d, variant, k2_dev, counts_dev ? counts_dev : nullptr, W, s);
}

int64_t epi3_pairs_workspace_bytes(const epi3_dataset *d, int32_t k, int64_t cand_cap) {
  return order_workspace_bytes(d, 2, k, cand_cap);
}
int epi3_scan_pairs(const epi3_dataset *d, int32_t k, int64_t cand_cap, void *ws_dev,
                    int64_t ws_bytes, void *stream) {
  return order_scan(d, 2, k, cand_cap, ws_dev, ws_bytes, stream);
}
int epi3_pairs_topk(const epi3_dataset *d, int32_t k, int64_t cand_cap, void *ws_dev,
                    epi3_pair_hit *hits_host, int32_t *n_out, void *stream) {
  return order_topk(d, 2, k, cand_cap, ws_dev, hits_host, n_out, stream);
}
int epi3_pairs_score_plane(const epi3_dataset *d, int32_t k, int64_t cand_cap, void *ws_dev,
                           float **plane_dev) {
  return order_score_plane(d, 2, k, cand_cap, ws_dev, plane_dev);
}

int64_t epi3_quads_workspace_bytes(const epi3_dataset *d, int32_t k, int64_t cand_cap) {
  return order_workspace_bytes(d, 4, k, cand_cap);
}
int epi3_scan_quads(const epi3_dataset *d, int32_t k, int64_t cand_cap, void *ws_dev,
                    int64_t ws_bytes, void *stream) {
  return order_scan(d, 4, k, cand_cap, ws_dev, ws_bytes, stream);
}
int epi3_quads_topk(const epi3_dataset *d, int32_t k, int64_t cand_cap, void *ws_dev,
                    epi3_quad_hit *hits_host, int32_t *n_out, void *stream) {
  return order_topk(d, 4, k, cand_cap, ws_dev, hits_host, n_out, stream);
}
int epi3_quads_score_plane(const epi3_dataset *d, int32_t k, int64_t cand_cap, void *ws_dev,
                           float **plane_dev) {
  return order_score_plane(d, 4, k, cand_cap, ws_dev, plane_dev);
}

int epi3_score_triplets(const epi3_dataset *d, const uint32_t *ijk_dev, int64_t n,
                        uint32_t *counts_dev, float *k2_f32_dev, double *k2_dev, void *stream) {
  if (!valid_dataset(d) || n < 0 || (n > 0 && !ijk_dev)) return EPI3_E_INVALID;
  if (d->layout != EPI3_LAYOUT_SPLIT) return EPI3_E_INVALID;
  HIP_OK(launch_score_triplets(*d, ijk_dev, n, counts_dev, k2_f32_dev, k2_dev,
                               static_cast<hipStream_t>(stream)));
  return EPI3_OK;
}

}  // extern "C"

namespace {

constexpr int kPermGroup = 64;  // phenotypes per matrix-core launch
constexpr int64_t kPermPassBytes = 4ll << 30;  // scratch for one pass of counted tiles

// Workspace of a batched scan.
struct BatchLayout {
  int n = 0, layout = 0, groups = 0;
  Job *jobs = nullptr;            // SPLIT
  PermJob *pjobs = nullptr;       // MASKED, one per group of 64 phenotypes
  PermJob *pjobs_alt = nullptr;   // the same with the second scratch buffer
  SelJob *sel = nullptr;
  SelState *st = nullptr;
  uint32_t *hist = nullptr;
  unsigned long long *queue = nullptr;
  const uint32_t **masks = nullptr;
  uint8_t *ph = nullptr;          // MASKED: [groups][64][S]
  int32_t *n1 = nullptr;          // MASKED: [groups][64]
  int32_t *case_pairs = nullptr;  // MASKED: [groups][Mp][Mp][64] uint2 (16-bit counts)
  int64_t *perm_prefix = nullptr; // MASKED: [M + 1]
  uint8_t *perm_scratch = nullptr;// MASKED: counts of one pass of tiles
  int64_t pass_tiles = 0;
  // MASKED, bounded selection (no score plane): every sample_stride-th tile
  // is scored first into a sample plane, whose k-th smallest score bounds
  // what the main pass appends to each job's list
  bool bounded = false;
  int64_t sample_stride = 0, sample_tiles = 0, sample_T = 0;
  float *sample = nullptr;        // [groups * 64][sample_T]
  SelJob *ssel = nullptr;         // [n] selection of the k-th sample score
  SelState *sst = nullptr;
  uint32_t *shist = nullptr;
  uint32_t *bkey = nullptr;       // [groups * 64][ccap]: the jobs' lists (ckey[x] points in)
  int64_t *brank = nullptr;
  epi3_hit *hits = nullptr;       // [sum k]
  std::vector<int64_t *> jprefix; // SPLIT, per job
  std::vector<float *> score;
  std::vector<int64_t *> cand;
  std::vector<uint32_t *> candkey;
  std::vector<CandRec *> rec;
  std::vector<uint64_t *> skey;   // sort buffers of jobs with capacities above kRankDirectMax
  std::vector<uint32_t *> sidx;
  std::vector<uint32_t *> ckey;
  std::vector<int64_t *> crank;
  std::vector<int64_t> cap, ccap, hit_off, T;
  std::vector<int> vsplit;        // SPLIT: count kernel of each job (EPI3_VARIANT_*)
  PlainJob *pjobs_plain = nullptr;// SPLIT: one record per matrix-core job
  int64_t *plain_begin = nullptr; // SPLIT: their global first tiles, per (type, JB) group
  uint8_t *plain_scratch = nullptr;
  int64_t plain_pass_tiles = 0;
  int64_t total_k = 0, total = 0;
};

bool same_dataset(const epi3_dataset *a, const epi3_dataset *b) {
  return a->planes == b->planes && a->n_snps == b->n_snps && a->n_samples == b->n_samples &&
         a->layout == b->layout;
}

int check_jobs(const epi3_job *jobs, int32_t n, int32_t variant) {
  if (!jobs || n <= 0) return EPI3_E_INVALID;
  if (variant < EPI3_VARIANT_AUTO || variant > EPI3_VARIANT_MFMA_FP4) return EPI3_E_INVALID;
  const int layout = jobs[0].d ? jobs[0].d->layout : -1;
  if (layout == EPI3_LAYOUT_MASKED && variant == EPI3_VARIANT_VALU) return EPI3_E_UNSUPPORTED;
  for (int x = 0; x < n; ++x) {
    const epi3_job &J = jobs[x];
    if (!valid_dataset(J.d) || J.k <= 0 || J.d->layout != layout) return EPI3_E_INVALID;
    if (layout == EPI3_LAYOUT_SPLIT && J.case_mask) return EPI3_E_INVALID;
    if (layout == EPI3_LAYOUT_SPLIT) {
      const int v = plain_variant(*J.d, variant);
      if (v < 0) return v;
    }
    if (layout == EPI3_LAYOUT_MASKED) {
      if (!J.case_mask || !J.d->bytes || !same_dataset(J.d, jobs[0].d)) return EPI3_E_INVALID;
      // counted cells and case pair tables are 16-bit
      if (J.d->n_samples > 65535 || !offsets32_ok(*J.d)) return EPI3_E_UNSUPPORTED;
    }
  }
  return EPI3_OK;
}

BatchLayout batch_layout(void *ws, const epi3_job *jobs, int32_t n, int64_t cand_cap,
                         int32_t variant) {
  BatchLayout L;
  L.n = n;
  L.layout = jobs[0].d->layout;
  Carver c(ws);
  L.sel = c.take<SelJob>(n);
  L.st = c.take<SelState>(n);
  L.hist = c.take<uint32_t>((int64_t)n * kHistBins);
  L.queue = c.take<unsigned long long>(8);  // tile counters (the phenotype count: one per XCD)
  L.hit_off.resize(n);
  for (int x = 0; x < n; ++x) {
    L.hit_off[x] = L.total_k;
    L.total_k += jobs[x].k;
  }
  L.hits = c.take<epi3_hit>(L.total_k);
  if (L.layout == EPI3_LAYOUT_SPLIT) {
    L.jobs = c.take<Job>(n);
    // per job: the vector-ALU kernel (all such jobs share one launch) or the
    // matrix cores (all jobs of one operand type and tile share one sequence
    // of launches through one scratch)
    L.vsplit.resize(n);
    std::map<std::pair<int, int>, int64_t> group_tiles;
    int n_mfma = 0;
    for (int x = 0; x < n; ++x) {
      const epi3_dataset &d = *jobs[x].d;
      L.vsplit[x] = plain_variant(d, variant);
      if ((L.vsplit[x] == EPI3_VARIANT_MFMA || L.vsplit[x] == EPI3_VARIANT_MFMA_FP4) &&
          epi3_n_triplets(d.n_snps) > 0) {
        ++n_mfma;
        const int JB = pick_JB(d, L.vsplit[x]);
        group_tiles[{L.vsplit[x], JB}] += host_plain_tiles(d.n_snps, JB);
      }
    }
    if (n_mfma > 0) {
      int64_t max_tiles = 0;
      for (const auto &kv : group_tiles) max_tiles = std::max(max_tiles, kv.second);
      L.pjobs_plain = c.take<PlainJob>(n);
      L.plain_begin = c.take<int64_t>((int64_t)n + (int64_t)group_tiles.size());
      L.plain_pass_tiles = std::max<int64_t>(
          1, std::min<int64_t>(max_tiles, pass_bytes(kPlainPassBytes) / kPlainTileScratch));
      L.plain_scratch = c.take<uint8_t>(2 * L.plain_pass_tiles * kPlainTileScratch);
    }
  } else {
    const epi3_dataset &d = *jobs[0].d;
    L.groups = (n + kPermGroup - 1) / kPermGroup;
    L.pjobs = c.take<PermJob>(L.groups);
    L.pjobs_alt = c.take<PermJob>(L.groups);
    L.masks = c.take<const uint32_t *>((int64_t)L.groups * kPermGroup);
    L.ph = c.take<uint8_t>((int64_t)L.groups * kPermGroup * d.byte_stride);
    L.n1 = c.take<int32_t>((int64_t)L.groups * kPermGroup);
    L.case_pairs = c.take<int32_t>((int64_t)L.groups * d.snp_stride * d.snp_stride * kPermGroup * 2);
    L.perm_prefix = c.take<int64_t>((int64_t)d.n_snps + 1);
    // counts of up to kPermPassBytes worth of tiles per pass
    const int64_t tiles = host_perm_tiles(d.n_snps);
    L.pass_tiles = std::max<int64_t>(
        1, std::min<int64_t>(tiles, pass_bytes(kPermPassBytes) / kPermTileScratch));
    int32_t max_k = 0;
    for (int x = 0; x < n; ++x) max_k = std::max(max_k, jobs[x].k);
    const int64_t T = epi3_n_triplets(d.n_snps);
    const int mode = batch_select_mode();
    if (T > 0 && (mode == EPI3_BATCH_SELECT_BOUNDED ||
                  (mode == EPI3_BATCH_SELECT_AUTO && T >= kBoundedMinTriplets))) {
      // about max(1024, 64 k) sample tiles (64 scores each), spread evenly
      // over the tile order
      const int64_t want = std::max<int64_t>(1024, 64 * (int64_t)max_k);
      const int64_t stride = std::max<int64_t>(1, tiles / want);
      if (host_perm_sample_valid(d.n_snps, stride) >= max_k) {
        L.bounded = true;
        L.sample_stride = stride;
        L.sample_tiles = (tiles + stride - 1) / stride;
        L.sample_T = L.sample_tiles * 64;
        L.sample = c.take<float>((int64_t)L.groups * kPermGroup * L.sample_T);
        L.ssel = c.take<SelJob>(n);
        L.sst = c.take<SelState>(n);
        L.shist = c.take<uint32_t>((int64_t)n * kHistBins);
      }
    }
    // two buffers: the count kernel of pass p + 1 runs while pass p is
    // scored; not needed where FP4 passes count and score in one kernel
    const bool fp4 = variant != EPI3_VARIANT_MFMA;
    if (!(L.bounded && fp4 && perm_fused_ok(d.n_samples + 2)))
      L.perm_scratch = c.take<uint8_t>(2 * L.pass_tiles * kPermTileScratch);
  }
  L.jprefix.resize(n);
  L.score.resize(n);
  L.cand.resize(n);
  L.candkey.resize(n);
  L.rec.resize(n);
  L.skey.resize(n);
  L.sidx.resize(n);
  L.ckey.resize(n);
  L.crank.resize(n);
  L.cap.resize(n);
  L.ccap.resize(n);
  L.T.resize(n);
  for (int x = 0; x < n; ++x) {
    L.T[x] = epi3_n_triplets(jobs[x].d->n_snps);
    L.cap[x] = default_cap(L.T[x], jobs[x].k, cand_cap);
    L.ccap[x] = compact_cap(L.T[x], L.cap[x]);
  }
  if (L.bounded) {
    // one list length for all jobs: the larger of the compacted-list size and
    // twice the expected count (the sample holds one score in sample_stride,
    // so about k sample_stride scores lie below its k-th), plus slack
    // (a size set by epi3_set_compact_cap is taken as it is)
    const bool fixed = compact_cap_override() > 0;
    int64_t cc = 0;
    for (int x = 0; x < n; ++x)
      cc = std::max(cc, fixed ? L.ccap[x]
                              : std::max(L.ccap[x], 2 * (int64_t)jobs[x].k * L.sample_stride + 65536));
    L.bkey = c.take<uint32_t>((int64_t)L.groups * kPermGroup * cc);
    L.brank = c.take<int64_t>((int64_t)L.groups * kPermGroup * cc);
    for (int x = 0; x < n; ++x) {
      L.ccap[x] = cc;
      L.score[x] = nullptr;
    }
  } else if (L.layout == EPI3_LAYOUT_MASKED) {
    // one block [n][T]: the matrix-core kernel addresses phenotype q at q * T
    float *all = c.take<float>((int64_t)n * L.T[0]);
    for (int x = 0; x < n; ++x) L.score[x] = all ? all + (int64_t)x * L.T[0] : nullptr;
  }
  for (int x = 0; x < n; ++x) {
    const epi3_dataset &d = *jobs[x].d;
    if (L.layout == EPI3_LAYOUT_SPLIT) {
      L.jprefix[x] = c.take<int64_t>((int64_t)d.n_snps + 1);
      L.score[x] = c.take<float>(L.T[x]);
    }
    L.cand[x] = c.take<int64_t>(L.cap[x]);
    L.candkey[x] = c.take<uint32_t>(L.cap[x]);
    L.rec[x] = c.take<CandRec>(L.cap[x]);
    L.skey[x] = c.take<uint64_t>(sort_len(L.cap[x]));
    L.sidx[x] = c.take<uint32_t>(sort_len(L.cap[x]));
    if (L.bounded) {
      L.ckey[x] = L.bkey ? L.bkey + (int64_t)x * L.ccap[x] : nullptr;
      L.crank[x] = L.brank ? L.brank + (int64_t)x * L.ccap[x] : nullptr;
    } else {
      L.ckey[x] = c.take<uint32_t>(L.ccap[x]);
      L.crank[x] = c.take<int64_t>(L.ccap[x]);
    }
  }
  L.total = c.size();
  return L;
}

// Enqueues the whole batched scan (no host synchronisation inside).
int enqueue_batched(const epi3_job *jobs, int32_t n, const BatchLayout &W, int32_t variant,
                    hipStream_t s) {
  const bool fp4 = variant != EPI3_VARIANT_MFMA;  // MASKED: AUTO and MFMA_FP4 use FP4
  AuxLease lease;  // second stream and events of the matrix-core passes
  if (lease.rc != EPI3_OK) return lease.rc;
  // selection state first: the count kernels write each job's key range into it
  std::vector<SelJob> sj(n);
  bool any_sample = false;
  for (int x = 0; x < n; ++x) {
    const epi3_dataset &d = *jobs[x].d;
    sj[x] = make_seljob(d, W.score[x], W.T[x], W.st + x, W.hist + (int64_t)x * kHistBins,
                        W.cand[x], W.candkey[x], W.rec[x], W.hits + W.hit_off[x], W.cap[x],
                        jobs[x].k, W.ckey[x], W.crank[x], W.ccap[x]);
    sj[x].skey = W.skey[x];
    sj[x].sidx = W.sidx[x];
    sj[x].sortP = sort_len(W.cap[x]);
    // bounded jobs have their list before the selection starts (no plane pass)
    if (W.bounded) sj[x].sample = 1;
    any_sample = any_sample || (sj[x].sample && sj[x].score);
    if (W.layout == EPI3_LAYOUT_MASKED) {
      const int g = x / kPermGroup, q = x % kPermGroup;
      sj[x].case_mask = jobs[x].case_mask;
      sj[x].case_pairs = W.case_pairs +
                         ((int64_t)g * d.snp_stride * d.snp_stride * kPermGroup + q) * 2;
      sj[x].case_stride = kPermGroup;
      sj[x].n1_dev = W.n1 + (int64_t)g * kPermGroup + q;
    }
  }
  HIP_OK(launch_write_seljobs(sj.data(), n, W.sel, s));
  HIP_OK(launch_init_select(W.sel, n, s));

  int64_t max_T = 0, max_cap = 0;
  int32_t max_k = 0;
  for (int x = 0; x < n; ++x) {
    max_T = std::max(max_T, W.T[x]);
    max_cap = std::max(max_cap, W.cap[x]);
    max_k = std::max(max_k, jobs[x].k);
  }

  if (W.layout == EPI3_LAYOUT_SPLIT) {
    // matrix-core jobs: one sequence of passes per (operand type, tile JB)
    // over all their tiles, the data sets with the most samples per tile
    // first so the queue ends on the cheapest tiles
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (int x = 0; x < n; ++x) {
      const int v = W.vsplit[x];
      if (v < 0) return v;
      if (v == EPI3_VARIANT_VALU || W.T[x] == 0) continue;
      groups[{v, pick_JB(*jobs[x].d, v)}].push_back(x);
    }
    int64_t rec = 0, beg = 0;
    for (auto &kv : groups) {
      std::vector<int> &xs = kv.second;
      std::stable_sort(xs.begin(), xs.end(), [&](int a, int b) {
        const epi3_dataset &da = *jobs[a].d, &db = *jobs[b].d;
        return da.words[0] + da.words[1] > db.words[0] + db.words[1];
      });
      std::vector<MfmaTask> tasks;
      for (int x : xs) tasks.push_back({jobs[x].d, W.score[x], nullptr, W.jprefix[x], &W.st[x].kmin});
      const MfmaBufs B{W.plain_scratch, W.plain_pass_tiles, W.pjobs_plain + rec,
                       W.plain_begin + beg, W.queue};
      const int rc = enqueue_count_mfma(tasks, kv.first.first == EPI3_VARIANT_MFMA_FP4,
                                        kv.first.second, B, s, lease.c);
      if (rc != EPI3_OK) return rc;
      rec += (int64_t)xs.size();
      beg += (int64_t)xs.size() + 1;
    }
    // vector-ALU jobs: one persistent launch over all their tiles; jobs with
    // the most samples per tile first so the queue ends on the cheapest tiles
    std::vector<int> order;
    for (int x = 0; x < n; ++x)
      if (W.vsplit[x] == EPI3_VARIANT_VALU) order.push_back(x);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      const epi3_dataset &da = *jobs[a].d, &db = *jobs[b].d;
      return da.words[0] + da.words[1] > db.words[0] + db.words[1];
    });
    const int nv = (int)order.size();
    int P_lo = 8, P_hi = 4;
    int32_t lf_len = 2;
    const float *lf32 = nullptr;
    for (int x : order) {
      P_lo = std::min(P_lo, pick_P(*jobs[x].d));
      P_hi = std::max(P_hi, pick_P(*jobs[x].d));
      if (jobs[x].d->n_samples + 2 > lf_len) {
        lf_len = jobs[x].d->n_samples + 2;
        lf32 = jobs[x].d->lf32;
      }
    }
    std::vector<Job> J(nv);
    int64_t begin = 0;
    for (int y = 0; y < nv; ++y) {
      const int x = order[y];
      J[y] = make_job(*jobs[x].d, W.score[x], nullptr, W.jprefix[x], &W.st[x].kmin,
                      pick_P(*jobs[x].d));
      J[y].tile_begin = begin;
      begin += J[y].n_tiles;
    }
    if (nv > 0) {
      HIP_OK(launch_write_jobs(J.data(), nv, W.jobs, s));
      HIP_OK(launch_tile_prefix(W.jobs, nv, s));
      HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(W.queue), 0u, 2, s));
    }
    if (begin > 0) {
      const int rc = timed(0, s, [&]() {
        return launch_count_valu(W.jobs, nv, begin, W.queue, lf32, lf_len, P_lo, P_hi, false, s) ==
                       hipSuccess
                   ? EPI3_OK
                   : EPI3_E_HIP;
      });
      if (rc != EPI3_OK) return rc;
    }
  } else {
    const epi3_dataset &d = *jobs[0].d;
    std::vector<const uint32_t *> masks((size_t)W.groups * kPermGroup, nullptr);
    for (int x = 0; x < n; ++x) masks[x] = jobs[x].case_mask;
    for (int x = n; x < (int)masks.size(); ++x) masks[x] = jobs[0].case_mask;  // never read
    HIP_OK(launch_write_ptrs(masks.data(), (int32_t)masks.size(), W.masks, s));
    const int64_t tiles = host_perm_tiles(d.n_snps);
    if (W.bounded) {
      // selection of each job's k-th smallest sample score
      std::vector<SelJob> ss(n);
      for (int x = 0; x < n; ++x)
        ss[x] = make_seljob(d, W.sample + (int64_t)x * W.sample_T, W.sample_T, W.sst + x,
                            W.shist + (int64_t)x * kHistBins, nullptr, nullptr, nullptr, nullptr,
                            1, jobs[x].k, nullptr, nullptr, 0);
      for (SelJob &j : ss) j.sample = 0;  // read as a whole
      HIP_OK(launch_write_seljobs(ss.data(), n, W.ssel, s));
      HIP_OK(launch_init_select(W.ssel, n, s));
    }
    for (int g = 0; g < W.groups; ++g) {
      const int Q = std::min(kPermGroup, n - g * kPermGroup);
      PermJob pj{};
      pj.bytes = static_cast<const uint8_t *>(fp4 ? d.nibbles : d.bytes);
      pj.ph = W.ph + (int64_t)g * kPermGroup * d.byte_stride;  // FP4 rows use the first half
      pj.tot_pairs = d.pairs;
      pj.case_pairs = W.case_pairs + (int64_t)g * d.snp_stride * d.snp_stride * kPermGroup * 2;
      pj.n1 = W.n1 + (int64_t)g * kPermGroup;
      pj.score = W.score[g * kPermGroup];
      pj.jprefix = W.perm_prefix;
      // no scratch where the passes count and score in one kernel
      uint8_t *scr[2] = {nullptr, nullptr};
      if (W.perm_scratch) {
        scr[0] = W.perm_scratch;
        scr[1] = W.perm_scratch + W.pass_tiles * kPermTileScratch;
      }
      pj.corners = reinterpret_cast<uint4 *>(scr[0]);
      pj.totals = scr[0] ? reinterpret_cast<uint4 *>(scr[0] + W.pass_tiles * 64 * 64 * 16) : nullptr;
      pj.n_tiles = tiles;
      pj.T = epi3_n_triplets(d.n_snps);
      pj.M = d.n_snps;
      pj.Mp = d.snp_stride;
      pj.S = fp4 ? d.byte_stride / 2 : d.byte_stride;
      pj.N = d.n_samples;
      pj.Q = Q;
      pj.Qp = kPermGroup;
      HIP_OK(launch_write_permjob(pj, W.pjobs + g, s));
      HIP_OK(launch_mask_bytes(W.masks + (int64_t)g * kPermGroup, Q, kPermGroup, d.n_samples,
                               d.byte_stride, const_cast<uint8_t *>(pj.ph),
                               const_cast<int32_t *>(pj.n1), fp4, s));
      HIP_OK(launch_case_pairs(static_cast<const uint32_t *>(d.planes), d.snp_stride, d.words[0],
                               W.masks + (int64_t)g * kPermGroup, Q, kPermGroup,
                               const_cast<int32_t *>(pj.case_pairs), s));
      if (g == 0) HIP_OK(launch_perm_prefix(W.pjobs + 0, s));
      hipStream_t s2 = lease.c->s2;
      hipEvent_t ev_start = lease.c->ev[0], ev_cnt[2] = {lease.c->ev[1], lease.c->ev[2]},
                 ev_fin[2] = {lease.c->ev[3], lease.c->ev[4]};
      PermJob pjb[2] = {pj, pj};
      pjb[1].corners = reinterpret_cast<uint4 *>(scr[1]);
      pjb[1].totals = scr[1] ? reinterpret_cast<uint4 *>(scr[1] + W.pass_tiles * 64 * 64 * 16) : nullptr;
      HIP_OK(launch_write_permjob(pjb[1], W.pjobs_alt + g, s));
      const PermJob *pdev[2] = {W.pjobs + g, W.pjobs_alt + g};
      // Passes over the tiles n * stride, n < n_all: pass p counts into scratch
      // buffer p % 2 on `s`; its finish kernel runs on the second stream while
      // `s` counts pass p + 1, and count p + 2 waits for finish p (same
      // buffer).  Events order the two streams (also when captured); the join
      // at the end puts everything on `s` again.
      auto passes = [&](int64_t n_all, int64_t stride, SelState *fst, PermOut out) -> int {
        if (fp4 && out.mode != kPermOutPlane && perm_fused_ok(d.n_samples + 2)) {
          // counted and scored by one persistent kernel over all the tiles:
          // no scratch, no second stream
          if (n_all <= 0) return EPI3_OK;
          HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(W.queue), 0u, 16, s));
          out.sample_base = 0;
          return timed(0, s, [&]() {
            return launch_count_score_perm(W.pjobs + g, 0, n_all, stride, W.queue, fst, d.lf32,
                                           d.n_samples + 2, out, s) == hipSuccess
                       ? EPI3_OK
                       : EPI3_E_HIP;
          });
        }
        if (!W.perm_scratch) return EPI3_E_INVALID;  // the layout and the passes disagree
        HIP_OK(hipEventRecord(ev_start, s));
        HIP_OK(hipStreamWaitEvent(s2, ev_start, 0));
        int p = 0;
        for (int64_t n0 = 0; n0 < n_all; n0 += W.pass_tiles, ++p) {
          const int64_t nn = std::min(W.pass_tiles, n_all - n0);
          const int b = p & 1;
          if (p >= 2) HIP_OK(hipStreamWaitEvent(s, ev_fin[b], 0));
          HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(W.queue), 0u, 16, s));
          int rc = timed(0, s, [&]() {
            return launch_count_mfma_perm(pdev[b], n0 * stride, nn, stride, W.queue, fp4, s) ==
                           hipSuccess
                       ? EPI3_OK
                       : EPI3_E_HIP;
          });
          if (rc != EPI3_OK) return rc;
          HIP_OK(hipEventRecord(ev_cnt[b], s));
          HIP_OK(hipStreamWaitEvent(s2, ev_cnt[b], 0));
          out.sample_base = n0;
          rc = timed(3, s2, [&]() {
            return launch_finish_perm(pdev[b], n0 * stride, nn, stride, fst, d.lf32,
                                      d.n_samples + 2, out, s2) == hipSuccess
                       ? EPI3_OK
                       : EPI3_E_HIP;
          });
          if (rc != EPI3_OK) return rc;
          HIP_OK(hipEventRecord(ev_fin[b], s2));
        }
        HIP_OK(hipEventRecord(ev_fin[0], s2));
        HIP_OK(hipStreamWaitEvent(s, ev_fin[0], 0));
        return EPI3_OK;
      };
      const int64_t x0 = (int64_t)g * kPermGroup;
      int rc = EPI3_OK;
      if (W.bounded) {
        // sample pass: every sample_stride-th tile scored into the sample
        // plane (slots of no triplet stay +inf), then each job's k-th sample
        // score sets the bound of its list
        float *smp = W.sample + x0 * W.sample_T;
        HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(smp), 0x7f800000u,
                               (int64_t)kPermGroup * W.sample_T, s));
        PermOut so{};
        so.mode = kPermOutSample;
        so.sample = smp;
        so.sample_T = W.sample_T;
        rc = passes(W.sample_tiles, W.sample_stride, W.sst + x0, so);
        if (rc != EPI3_OK) return rc;
        HIP_OK(launch_select_kth(W.ssel + x0, Q, W.sample_T, s));
        HIP_OK(launch_sample_bound(W.sel + x0, W.ssel + x0, Q, s));
        PermOut bo{};
        bo.mode = kPermOutBounded;
        bo.ckey = W.ckey[x0];
        bo.crank = W.crank[x0];
        bo.ccap = W.ccap[x0];
        rc = passes(tiles, 1, W.st + x0, bo);
      } else {
        PermOut po{};
        po.mode = kPermOutPlane;
        rc = passes(tiles, 1, W.st + x0, po);
      }
      if (rc != EPI3_OK) return rc;
    }
  }
  // bounded jobs' passes read their lists only: size the grids for those
  const int64_t sel_T = W.bounded ? W.ccap[0] : max_T;
  return timed(1, s, [&]() {
    return launch_select(W.sel, n, sel_T, max_cap, max_k, any_sample, s) == hipSuccess ? EPI3_OK
                                                                                    : EPI3_E_HIP;
  });
}

bool timing_on() {
  Timing &t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  return t.on;
}

// Graphs cached per job signature.
struct GraphCache {
  std::mutex mu;
  std::map<std::vector<uint64_t>, hipGraphExec_t> exec;
  hipStream_t capture = nullptr;
};
GraphCache &graphs() {
  static GraphCache g;
  return g;
}

std::vector<uint64_t> signature(const epi3_job *jobs, int32_t n, int32_t variant, int64_t cap,
                                void *ws, int64_t ws_bytes) {
  std::vector<uint64_t> sig;
  sig.push_back((uint64_t)n);
  sig.push_back((uint64_t)variant);
  sig.push_back((uint64_t)cap);
  sig.push_back((uint64_t)(uintptr_t)ws);
  sig.push_back((uint64_t)ws_bytes);
  // tile rules, pass bytes and the compacted-list size change the captured work
  sig.push_back(settings_gen());
  for (int x = 0; x < n; ++x) {
    const epi3_dataset &d = *jobs[x].d;
    const uint64_t *raw = reinterpret_cast<const uint64_t *>(&d);
    for (size_t w = 0; w < sizeof(epi3_dataset) / 8; ++w) sig.push_back(raw[w]);
    sig.push_back((uint64_t)(uintptr_t)jobs[x].case_mask);
    sig.push_back((uint64_t)jobs[x].k);
  }
  return sig;
}

}  // namespace

extern "C" {

int64_t epi3_batched_workspace_bytes(const epi3_job *jobs, int32_t n_jobs, int32_t variant,
                                     int64_t cand_cap) {
  const int rc = check_jobs(jobs, n_jobs, variant);
  if (rc != EPI3_OK) return rc;
  return batch_layout(nullptr, jobs, n_jobs, cand_cap, variant).total;
}

int epi3_batched_score_plane(const epi3_job *jobs, int32_t n_jobs, int32_t variant,
                             int64_t cand_cap, void *ws_dev, int32_t job, float **plane_dev) {
  const int rc = check_jobs(jobs, n_jobs, variant);
  if (rc != EPI3_OK) return rc;
  if (!ws_dev || !plane_dev || job < 0 || job >= n_jobs) return EPI3_E_INVALID;
  const BatchLayout W = batch_layout(ws_dev, jobs, n_jobs, cand_cap, variant);
  if (!W.score[job]) return EPI3_E_UNSUPPORTED;
  *plane_dev = W.score[job];
  return EPI3_OK;
}

int epi3_batched_bound_list(const epi3_job *jobs, int32_t n_jobs, int32_t variant,
                            int64_t cand_cap, void *ws_dev, int32_t job, uint32_t **keys_dev,
                            int64_t **ranks_dev, int64_t *count, float *bound, void *stream) {
  const int rc = check_jobs(jobs, n_jobs, variant);
  if (rc != EPI3_OK) return rc;
  if (!ws_dev || !keys_dev || !ranks_dev || !count || !bound || job < 0 || job >= n_jobs)
    return EPI3_E_INVALID;
  const BatchLayout W = batch_layout(ws_dev, jobs, n_jobs, cand_cap, variant);
  if (!W.bounded) return EPI3_E_UNSUPPORTED;
  hipStream_t s = static_cast<hipStream_t>(stream);
  SelState st;
  HIP_OK(hipMemcpyAsync(&st, W.st + job, sizeof(st), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  *keys_dev = W.ckey[job];
  *ranks_dev = W.crank[job];
  *count = std::min<int64_t>((int64_t)st.cn, W.ccap[job]);
  *bound = st.ub;
  return EPI3_OK;
}

int epi3_scan_batched(const epi3_job *jobs, int32_t n_jobs, int32_t variant, int64_t cand_cap,
                      void *ws_dev, int64_t ws_bytes, epi3_hit *hits_host, int32_t *n_out_host,
                      void *stream) {
  int rc = check_jobs(jobs, n_jobs, variant);
  if (rc != EPI3_OK) return rc;
  if (!ws_dev || !hits_host || !n_out_host) return EPI3_E_INVALID;
  if (reinterpret_cast<uintptr_t>(ws_dev) % kAlign) return EPI3_E_INVALID;
  BatchLayout W = batch_layout(ws_dev, jobs, n_jobs, cand_cap, variant);
  if (ws_bytes < W.total) return EPI3_E_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);

  GraphCache &G = graphs();
  hipGraphExec_t exec = nullptr;
  if (timing_on()) {
    // measurement mode: run the same sequence eagerly so each kernel is timed
    rc = timed(2, s, [&]() { return enqueue_batched(jobs, n_jobs, W, variant, s); });
    if (rc != EPI3_OK) return rc;
  } else {
    std::lock_guard<std::mutex> lk(G.mu);
    const auto sig = signature(jobs, n_jobs, variant, cand_cap, ws_dev, ws_bytes);
    auto it = G.exec.find(sig);
    if (it != G.exec.end()) {
      exec = it->second;
    } else {
      if (!G.capture) HIP_OK(hipStreamCreateWithFlags(&G.capture, hipStreamNonBlocking));
      HIP_OK(hipStreamBeginCapture(G.capture, hipStreamCaptureModeRelaxed));
      rc = enqueue_batched(jobs, n_jobs, W, variant, G.capture);
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(G.capture, &graph);
      if (rc != EPI3_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc != EPI3_OK ? rc : EPI3_E_HIP;
      }
      const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) return EPI3_E_HIP;
      G.exec[sig] = exec;
    }
    if (hipGraphLaunch(exec, s) != hipSuccess) return EPI3_E_HIP;
  }

  std::vector<SelState> st(n_jobs);
  HIP_OK(hipMemcpyAsync(st.data(), W.st, sizeof(SelState) * n_jobs, hipMemcpyDeviceToHost, s));
  std::vector<int32_t> status(n_jobs, 0);
  for (int x = 0; x < n_jobs; ++x)
    HIP_OK(hipMemcpyAsync(&status[x], jobs[x].d->status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(hits_host, W.hits, sizeof(epi3_hit) * W.total_k, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  int worst = EPI3_OK;
  for (int x = 0; x < n_jobs; ++x) {
    n_out_host[x] = (int32_t)st[x].keff;
    if (status[x] & 1) {
      n_out_host[x] = 0;
      worst = EPI3_E_GENOTYPE;
    } else if (st[x].done == 3u) {
      // the bounded list overflowed: 16 x cand_cap entries hold it on a retry
      const int64_t need = std::max<int64_t>((int64_t)((st[x].cn + 15) / 16), W.cap[x] + 1);
      n_out_host[x] = -(int32_t)std::min<int64_t>(need, 0x7fffffff);
      if (worst == EPI3_OK) worst = EPI3_E_CAPACITY;
    } else if ((int64_t)st[x].ncand > W.cap[x]) {
      n_out_host[x] = -(int32_t)std::min<unsigned long long>(st[x].ncand, 0x7fffffffull);
      if (worst == EPI3_OK) worst = EPI3_E_CAPACITY;
    }
  }
  return worst;
}

int epi3_init(void) {
  {
    AuxLease lease;  // one idle context in the pool from now on
    if (lease.rc != EPI3_OK) return lease.rc;
  }
  {
    const int rc = static_scratch_ptr(nullptr);  // epi3_scan_topk_static's workspace
    if (rc != EPI3_OK) return rc;
  }
  GraphCache &G = graphs();
  std::lock_guard<std::mutex> lk(G.mu);
  if (!G.capture) HIP_OK(hipStreamCreateWithFlags(&G.capture, hipStreamNonBlocking));
  return EPI3_OK;
}

void epi3_release(void) {
  {
    AuxPool &p = aux_pool();
    std::lock_guard<std::mutex> lk(p.mu);
    for (AuxCtx *c : p.idle) aux_destroy(c);
    p.idle.clear();
  }
  GraphCache &G = graphs();
  std::lock_guard<std::mutex> lk(G.mu);
  for (auto &kv : G.exec) (void)hipGraphExecDestroy(kv.second);
  G.exec.clear();
  if (G.capture) {
    (void)hipStreamDestroy(G.capture);
    G.capture = nullptr;
  }
}

int epi3_perm_pvalue(double observed_k2, const double *perm_min_k2, int32_t n_perm, double *p_out) {
  if (!perm_min_k2 || !p_out || n_perm < 1 || observed_k2 != observed_k2) return EPI3_E_INVALID;
  int64_t hits = 0;
  for (int32_t q = 0; q < n_perm; ++q) {
    if (perm_min_k2[q] != perm_min_k2[q]) return EPI3_E_INVALID;
    hits += perm_min_k2[q] <= observed_k2;
  }
  *p_out = (double)(1 + hits) / (double)(n_perm + 1);
  return EPI3_OK;
}

int epi3_tile_rule(int32_t variant, int32_t min_snps, int32_t min_samples, int32_t tile) {
  if (min_snps < 0 || min_samples < 0) return EPI3_E_INVALID;
  bool ok = false;
  if (variant == EPI3_VARIANT_VALU) ok = tile == 4 || tile == 8;
  if (variant == EPI3_VARIANT_MFMA || variant == EPI3_VARIANT_MFMA_FP4)
    ok = tile == 2 || tile == 4 || tile == 8;
  if (variant == EPI3_VARIANT_AUTO)
    ok = tile == EPI3_VARIANT_VALU || tile == EPI3_VARIANT_MFMA || tile == EPI3_VARIANT_MFMA_FP4;
  if (!ok) return EPI3_E_INVALID;
  Tiles &t = tiles();
  std::lock_guard<std::mutex> g(t.mu);
  for (TileRule &r : t.rules) {
    if (r.variant == variant && r.min_snps == min_snps && r.min_samples == min_samples) {
      r.tile = tile;
      ++t.gen;
      return EPI3_OK;
    }
  }
  t.rules.push_back({variant, min_snps, min_samples, tile});
  ++t.gen;
  return EPI3_OK;
}

void epi3_tile_rules_clear(void) {
  Tiles &t = tiles();
  std::lock_guard<std::mutex> g(t.mu);
  t.rules.clear();
  ++t.gen;
}

int32_t epi3_tile_for(const epi3_dataset *d, int32_t variant) {
  if (!valid_dataset(d)) return EPI3_E_INVALID;
  if (variant == EPI3_VARIANT_AUTO) return plain_variant(*d, variant);
  if (variant == EPI3_VARIANT_VALU) return pick_P(*d);
  if (variant == EPI3_VARIANT_MFMA || variant == EPI3_VARIANT_MFMA_FP4) return pick_JB(*d, variant);
  return EPI3_E_INVALID;
}

int epi3_set_compact_cap(int64_t n) {
  if (n < 0) return EPI3_E_INVALID;
  Tiles &t = tiles();
  std::lock_guard<std::mutex> g(t.mu);
  t.compact_cap = n;
  ++t.gen;
  return EPI3_OK;
}

int epi3_set_batch_select(int32_t mode) {
  if (mode < EPI3_BATCH_SELECT_AUTO || mode > EPI3_BATCH_SELECT_BOUNDED) return EPI3_E_INVALID;
  Tiles &t = tiles();
  std::lock_guard<std::mutex> g(t.mu);
  t.batch_select = mode;
  ++t.gen;
  return EPI3_OK;
}

int epi3_set_scan_select(int32_t mode) {
  if (mode < EPI3_SCAN_SELECT_AUTO || mode > EPI3_SCAN_SELECT_BOUNDED) return EPI3_E_INVALID;
  Tiles &t = tiles();
  std::lock_guard<std::mutex> g(t.mu);
  t.scan_select = mode;
  ++t.gen;
  return EPI3_OK;
}

int epi3_set_pass_bytes(int64_t bytes) {
  if (bytes < 0) return EPI3_E_INVALID;
  Tiles &t = tiles();
  std::lock_guard<std::mutex> g(t.mu);
  t.pass_bytes = bytes;
  ++t.gen;
  return EPI3_OK;
}

void epi3_timing_enable(int enable) {
  Timing &t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  t.on = enable != 0;
}

int epi3_timing_query(int32_t which, double *ms, int64_t *launches) {
  if (which < 0 || which > 4 || !ms || !launches) return EPI3_E_INVALID;
  Timing &t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  double sum = 0.0;
  for (auto &p : t.rec[which]) {
    if (hipEventSynchronize(p.second) != hipSuccess) return EPI3_E_HIP;
    float x = 0.f;
    if (hipEventElapsedTime(&x, p.first, p.second) != hipSuccess) return EPI3_E_HIP;
    sum += x;
  }
  *ms = sum;
  *launches = (int64_t)t.rec[which].size();
  return EPI3_OK;
}

void epi3_timing_reset(void) {
  Timing &t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  for (auto &r : t.rec) {
    for (auto &p : r) {
      (void)hipEventSynchronize(p.second);
      t.pool.push_back(p.first);
      t.pool.push_back(p.second);
    }
    r.clear();
  }
}

}  // extern "C"

static double order_error_bound(int order, int32_t n_samples) {
  return order == 2 ? epi3_k2_error_bound_pairs(n_samples) : epi3_k2_error_bound_quads(n_samples);
}
