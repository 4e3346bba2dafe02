// hs_lib.hip -- host side of the C ABI declared in include/hs.h: database
// loading and packing, argument checking, kernel launches and result
// marshalling.  Everything the search computes runs in the kernels of the
// headers included below.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hs.h"
#include "device_common.hpp"
#include "score_kernels.hpp"
#include "topk_kernels.hpp"
#include "traceback_kernels.hpp"
#include "sw_kernels.hpp"
#include "threshold_kernels.hpp"
#include "align_kernels.hpp"

using namespace hs;

static_assert(sizeof(hs_hit) == sizeof(DevHit), "hit layout");
static_assert(sizeof(hs_aln) == sizeof(DevAln), "alignment layout");
static_assert(kAlMaxLen == HS_MAX_ALIGN, "pairwise length limit");

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(HS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// BLOSUM62 (Henikoff & Henikoff 1992), alphabet ARNDCQEGHILKMFPSTWYVBZX*.
const int8_t kBlosum62[kNsym * kNsym] = {
    4, -1, -2, -2, 0, -1, -1, 0, -2, -1, -1, -1, -1, -2, -1, 1, 0, -3, -2, 0, -2, -1, 0, -4,
    -1, 5, 0, -2, -3, 1, 0, -2, 0, -3, -2, 2, -1, -3, -2, -1, -1, -3, -2, -3, -1, 0, -1, -4,
    -2, 0, 6, 1, -3, 0, 0, 0, 1, -3, -3, 0, -2, -3, -2, 1, 0, -4, -2, -3, 3, 0, -1, -4,
    -2, -2, 1, 6, -3, 0, 2, -1, -1, -3, -4, -1, -3, -3, -1, 0, -1, -4, -3, -3, 4, 1, -1, -4,
    0, -3, -3, -3, 9, -3, -4, -3, -3, -1, -1, -3, -1, -2, -3, -1, -1, -2, -2, -1, -3, -3, -2, -4,
    -1, 1, 0, 0, -3, 5, 2, -2, 0, -3, -2, 1, 0, -3, -1, 0, -1, -2, -1, -2, 0, 3, -1, -4,
    -1, 0, 0, 2, -4, 2, 5, -2, 0, -3, -3, 1, -2, -3, -1, 0, -1, -3, -2, -2, 1, 4, -1, -4,
    0, -2, 0, -1, -3, -2, -2, 6, -2, -4, -4, -2, -3, -3, -2, 0, -2, -2, -3, -3, -1, -2, -1, -4,
    -2, 0, 1, -1, -3, 0, 0, -2, 8, -3, -3, -1, -2, -1, -2, -1, -2, -2, 2, -3, 0, 0, -1, -4,
    -1, -3, -3, -3, -1, -3, -3, -4, -3, 4, 2, -3, 1, 0, -3, -2, -1, -3, -1, 3, -3, -3, -1, -4,
    -1, -2, -3, -4, -1, -2, -3, -4, -3, 2, 4, -2, 2, 0, -3, -2, -1, -2, -1, 1, -4, -3, -1, -4,
    -1, 2, 0, -1, -3, 1, 1, -2, -1, -3, -2, 5, -1, -3, -1, 0, -1, -3, -2, -2, 0, 1, -1, -4,
    -1, -1, -2, -3, -1, 0, -2, -3, -2, 1, 2, -1, 5, 0, -2, -1, -1, -1, -1, 1, -3, -1, -1, -4,
    -2, -3, -3, -3, -2, -3, -3, -3, -1, 0, 0, -3, 0, 6, -4, -2, -2, 1, 3, -1, -3, -3, -1, -4,
    -1, -2, -2, -1, -3, -1, -1, -2, -2, -3, -3, -1, -2, -4, 7, -1, -1, -4, -3, -2, -2, -1, -2, -4,
    1, -1, 1, 0, -1, 0, 0, 0, -1, -2, -2, 0, -1, -2, -1, 4, 1, -3, -2, -2, 0, 0, 0, -4,
    0, -1, 0, -1, -1, -1, -1, -2, -2, -1, -1, -1, -1, -2, -1, 1, 5, -2, -2, 0, -1, -1, 0, -4,
    -3, -3, -4, -4, -2, -2, -3, -2, -2, -3, -2, -3, -1, 1, -4, -3, -2, 11, 2, -3, -4, -3, -2, -4,
    -2, -2, -2, -3, -2, -1, -2, -3, 2, -1, -1, -2, -1, 3, -3, -2, -2, 2, 7, -1, -3, -2, -1, -4,
    0, -3, -3, -3, -1, -2, -2, -3, -3, 3, 1, -2, 1, -1, -2, -2, 0, -3, -1, 4, -3, -2, -1, -4,
    -2, -1, 3, 4, -3, 0, 1, -1, 0, -3, -4, 0, -3, -3, -2, 0, -1, -4, -3, -3, 4, 1, -1, -4,
    -1, 0, 0, 1, -3, 3, 4, -2, 0, -3, -3, 1, -1, -3, -1, 0, -1, -3, -2, -2, 1, 4, -1, -4,
    0, -1, -1, -1, -2, -1, -1, -1, -1, -1, -1, -1, -1, -1, -2, 0, 0, -2, -1, -1, -1, -1, -1, -4,
    -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, 1,
};

const char kAlphabet[] = "ARNDCQEGHILKMFPSTWYVBZX*";

// ASCII -> code, -1 for bytes outside the alphabet.
struct CodeTable {
    int8_t t[256];
    CodeTable() {
        for (int i = 0; i < 256; ++i) t[i] = -1;
        for (int i = 0; i < kNsym; ++i) {
            const unsigned char c = (unsigned char)kAlphabet[i];
            t[c] = (int8_t)i;
            if (c >= 'A' && c <= 'Z') t[c - 'A' + 'a'] = (int8_t)i;
        }
        for (char c : {'J', 'O', 'U'}) {
            t[(unsigned char)c] = 22;
            t[(unsigned char)(c - 'A' + 'a')] = 22;
        }
    }
};
const CodeTable kCodes;

__constant__ int8_t c_codes[256];

}  // namespace

namespace hs_internal {
void set_error(const std::string& msg) { g_err = msg; }
}  // namespace hs_internal

// --------------------------------------------------------------------------
// database image
// --------------------------------------------------------------------------
struct hs_db {
    int64_t n_targets = 0;
    int64_t n_residues = 0;
    uint8_t* d_letters = nullptr;   // codes, index order, kLetterPad readable bytes after
    uint8_t* d_letters5 = nullptr;  // the same letters at 5 bits each (built on request)
    int32_t letter_bits = 8;        // image the one-query scoring kernel reads
    int64_t* d_offsets = nullptr;
    int32_t* d_lens = nullptr;
    int32_t* d_order = nullptr;     // longest first
    PairRec* d_recs = nullptr;      // (index, length, offset) in hand-out order
    int64_t n_queue = 0;            // hand-out positions (targets plus padding)
    int32_t median_len = 0;         // median target length (0 for an empty database)
    std::vector<int32_t> lens_desc; // target lengths, longest first (host copy)
    int64_t device_bytes = 0;

    DbView view() const {
        DbView v;
        v.letters = d_letters;
        v.offsets = d_offsets;
        v.lens = d_lens;
        v.order = d_order;
        v.n = (int32_t)n_targets;
        return v;
    }
};

// Encodes ASCII letters to alphabet codes in place; flags bytes outside the
// alphabet.
__global__ __launch_bounds__(256) void k_encode(uint8_t* __restrict__ letters, int64_t n,
                                                int32_t* err) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = c_codes[letters[i]];
        if (c < 0) atomicOr(err, 1);
        letters[i] = (uint8_t)(c < 0 ? 0 : c);
    }
}

// 5-bit image: letter i at bits 5i .. 5i + 4 of a little-endian stream of
// dwords; thread w writes dword w.  Letters past the last one read as the
// zero-row code, like the byte image's padding.
__global__ __launch_bounds__(256) void k_pack5(const uint8_t* __restrict__ letters, int64_t n,
                                               int64_t n_words, uint32_t* __restrict__ out) {
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < n_words;
         w += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b0 = 32 * w;                 // first bit of the dword
        uint32_t v = 0;
        for (int64_t i = b0 / 5; i * 5 < b0 + 32; ++i) {
            const uint32_t c = i < n ? letters[i] : (uint32_t)kZeroRow;
            const int64_t b = 5 * i;
            v |= b >= b0 ? c << (uint32_t)(b - b0) : c >> (uint32_t)(b0 - b);
        }
        out[w] = v;
    }
}

// Uploads and downloads of a batch between device memory and its pinned
// host mirrors (coherent host memory, which the device reads and writes
// directly, never caching it): segment s copies len[s] bytes from src +
// soff[s] to dst + doff[s] (offsets and lengths multiples of 16).  A kernel
// rather than a copy-engine transfer: served batches are small, and
// hipMemcpyAsync of them now and then blocked the host for milliseconds.
struct CopySegs {
    int64_t soff[3], doff[3];
    int64_t len[3];
    int32_t n;
};
__global__ __launch_bounds__(256) void k_copy_segs(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                   CopySegs sg) {
    for (int32_t k = 0; k < sg.n; ++k) {
        const int64_t so = sg.soff[k] >> 4, d = sg.doff[k] >> 4, n = sg.len[k] >> 4;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * blockDim.x)
            dst[d + i] = src[so + i];
    }
}

namespace {

void free_db(hs_db* db) {
    if (!db) return;
    (void)hipFree(db->d_letters);
    (void)hipFree(db->d_letters5);
    (void)hipFree(db->d_offsets);
    (void)hipFree(db->d_lens);
    (void)hipFree(db->d_order);
    (void)hipFree(db->d_recs);
    delete db;
}

template <class T>
int dev_alloc(T** p, size_t count, int64_t* acc) {
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (hipMalloc((void**)p, bytes) != hipSuccess) {
        *p = nullptr;
        return fail(HS_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    if (acc) *acc += (int64_t)bytes;
    return HS_OK;
}

int check_params(const hs_params* p) {
    if (!p) return fail(HS_EINVAL, "params is NULL");
    auto bad_pen = [](int32_t v) { return v < 0 || v > HS_MAX_PENALTY; };
    if (bad_pen(p->gop) || bad_pen(p->gep) || bad_pen(p->pgp))
        return fail(HS_EINVAL, "gap penalties must lie in [0, HS_MAX_PENALTY]");
    auto bad_fac = [](int32_t v) { return v < 0 || v > 65536; };
    if (bad_fac(p->lfactor_q16) || bad_fac(p->sfactor_q16) || bad_fac(p->minfactor_q16))
        return fail(HS_EINVAL, "factors must lie in [0, 65536] (Q16)");
    if (p->rounds < 1 || p->rounds > 1024) return fail(HS_EINVAL, "rounds must lie in [1, 1024]");
    if (p->matrix) {
        int mn = 127, mx = -128;
        for (int i = 0; i < kNsym * kNsym; ++i) {
            mn = std::min<int>(mn, p->matrix[i]);
            mx = std::max<int>(mx, p->matrix[i]);
        }
        if (mx - mn > 15) return fail(HS_EINVAL, "matrix entries must span at most 15");
    }
    return HS_OK;
}

KParams kparams(const hs_params* p) {
    KParams k;
    k.gop = p->gop;
    k.gep = p->gep;
    k.pgp = p->pgp;
    k.lfactor = (uint32_t)p->lfactor_q16;
    k.sfactor = (uint32_t)p->sfactor_q16;
    k.minfactor = (uint32_t)p->minfactor_q16;
    k.rounds = p->rounds;
    k.min_score = p->min_score;
    k.seed = p->seed;
    return k;
}

KMatrix kmatrix(const hs_params* p) {
    KMatrix m;
    std::memcpy(m.m, p->matrix ? p->matrix : kBlosum62, sizeof(m.m));
    return m;
}

// Offset that makes every matrix entry a byte in 0..15.
int32_t matrix_bias(const KMatrix& m) {
    int mn = 127;
    for (int i = 0; i < kNsym * kNsym; ++i) mn = std::min<int>(mn, m.m[i]);
    return -mn;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Per-query workspace carve-up.
struct QueryWs {
    int32_t* scores;
    int32_t* rounds;
    uint64_t* draws;
    uint32_t* queue;
    TopkState* topk;
    uint32_t* hist;
    uint64_t* keys;
    TopkWs tw() const {
        TopkWs t;
        t.st = topk;
        t.hist = hist;
        t.keys = keys;
        return t;
    }
};

size_t query_ws_bytes(int64_t n_targets, int64_t n_queue, int32_t k) {
    const size_t n = (size_t)std::max<int64_t>(n_targets, 1);
    const size_t nq = (size_t)std::max<int64_t>(n_queue, 1);
    (void)k;
    return 2 * align_up(sizeof(int32_t) * n) + align_up(sizeof(uint64_t) * 8 * nq) + kAlign +
           align_up(sizeof(TopkState)) + align_up(sizeof(uint32_t) * kWinBins) +
           align_up(sizeof(uint64_t) * kSortCap);
}

QueryWs carve(void* ws, int64_t n_targets, int64_t n_queue) {
    const size_t n = (size_t)std::max<int64_t>(n_targets, 1);
    const size_t nq = (size_t)std::max<int64_t>(n_queue, 1);
    char* p = (char*)ws;
    QueryWs q;
    q.scores = (int32_t*)p;
    p += align_up(sizeof(int32_t) * n);
    q.rounds = (int32_t*)p;
    p += align_up(sizeof(int32_t) * n);
    q.draws = (uint64_t*)p;
    p += align_up(sizeof(uint64_t) * 8 * nq);
    q.queue = (uint32_t*)p;
    p += kAlign;
    q.topk = (TopkState*)p;
    p += align_up(sizeof(TopkState));
    q.hist = (uint32_t*)p;
    p += align_up(sizeof(uint32_t) * kWinBins);
    q.keys = (uint64_t*)p;
    return q;
}

int check_search_args(const hs_db* db, int32_t qlen, const hs_params* p, int32_t k,
                      int32_t n_aln) {
    if (!db) return fail(HS_EINVAL, "db is NULL");
    if (qlen < 1 || qlen > HS_MAX_QUERY) return fail(HS_EINVAL, "qlen must lie in [1, HS_MAX_QUERY]");
    if (k < 1 || k > HS_MAX_K) return fail(HS_EINVAL, "k must lie in [1, HS_MAX_K]");
    if (n_aln < 0 || n_aln > k) return fail(HS_EINVAL, "n_aln must lie in [0, k]");
    return check_params(p);
}

int check_threshold_args(const hs_db* db, int32_t qlen, const hs_params* p, int64_t cap,
                         int32_t n_aln) {
    if (!db) return fail(HS_EINVAL, "db is NULL");
    if (qlen < 1 || qlen > HS_MAX_QUERY) return fail(HS_EINVAL, "qlen must lie in [1, HS_MAX_QUERY]");
    if (cap < 0) return fail(HS_EINVAL, "cap must be >= 0");
    if (n_aln < 0 || n_aln > HS_MAX_K) return fail(HS_EINVAL, "n_aln must lie in [0, HS_MAX_K]");
    return check_params(p);
}

// Kernels' LDS limits and occupancies are functions of (device, kernel,
// threads, LDS bytes) only; a batch asks the same questions for every query
// set, so the answers are kept (for every thread of the process).
struct LdsLimit {
    int dev;
    const void* fn;
    size_t bytes;
};
struct Occupancy {
    int dev;
    const void* fn;
    int threads;
    size_t lds;
    int per_cu;
};
// Fixed capacity, so that asking allocates nothing (hs_search_dev_noalloc
// relies on it); once full, answers are asked of the runtime again instead
// of kept.
template <class T, int N>
struct FixedCache {
    T v[N];
    int n = 0;
    T* begin() { return v; }
    T* end() { return v + n; }
    void push_back(const T& x) {
        if (n < N) v[n++] = x;
    }
};
std::mutex g_kernel_info_mu;
FixedCache<LdsLimit, 256> g_lds_limits;
FixedCache<Occupancy, 512> g_occupancies;

int current_device() {
    int dev = 0;
    return hipGetDevice(&dev) == hipSuccess ? dev : -1;
}

int set_lds_limit(const void* fn, size_t bytes) {
    if (bytes <= 64 * 1024) return HS_OK;
    const int dev = current_device();
    std::lock_guard<std::mutex> lock(g_kernel_info_mu);
    for (const LdsLimit& l : g_lds_limits)
        if (l.dev == dev && l.fn == fn && l.bytes >= bytes) return HS_OK;
    HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    for (LdsLimit& l : g_lds_limits)
        if (l.dev == dev && l.fn == fn) {
            l.bytes = bytes;
            return HS_OK;
        }
    g_lds_limits.push_back(LdsLimit{dev, fn, bytes});
    return HS_OK;
}

// Workgroups of fn resident per compute unit (the LDS limit already set).
int occupancy(const void* fn, int threads, size_t lds, int* per_cu) {
    const int dev = current_device();
    {
        std::lock_guard<std::mutex> lock(g_kernel_info_mu);
        for (const Occupancy& o : g_occupancies)
            if (o.dev == dev && o.fn == fn && o.threads == threads && o.lds == lds) {
                *per_cu = o.per_cu;
                return HS_OK;
            }
    }
    int v = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, fn, threads, lds));
    std::lock_guard<std::mutex> lock(g_kernel_info_mu);
    g_occupancies.push_back(Occupancy{dev, fn, threads, lds, v});
    *per_cu = v;
    return HS_OK;
}

size_t device_lds_limit() {
    static size_t lim = 0;
    if (!lim) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            v > 0)
            lim = (size_t)v;
        else
            lim = 64 * 1024;
    }
    return lim;
}

int device_cus() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1)
        return 256;
    return v;
}

// Wavefronts per workgroup beside a profile region of prof_bytes: as many as
// fit in LDS (at most 8; 0 if none), each with its WaveLds record.
int fit_waves(size_t prof_bytes) {
    for (int w = kWaves; w >= 1; --w)
        if (prof_bytes + sizeof(WaveLds) * w + 16 <= device_lds_limit()) return w;
    return 0;
}

// Profile layout of a one-query launch: four copies when they fit beside a
// full workgroup, else one copy (waves: the workgroup's wavefronts).
struct QueryLayout {
    int copies, waves;
    size_t lds;
};
int query_layout(int32_t qlen, QueryLayout* L) {
    const size_t p4 = (size_t)profile_region_bytes(qlen, 4);
    const size_t p1 = (size_t)profile_region_bytes(qlen, 1);
    if (fit_waves(p4) == kWaves) {
        L->copies = 4;
        L->waves = kWaves;
        L->lds = p4 + sizeof(WaveLds) * kWaves;
        return HS_OK;
    }
    L->copies = 1;
    L->waves = fit_waves(p1);
    if (L->waves < 1) return fail(HS_EINVAL, "query too long for the device's LDS");
    L->lds = p1 + sizeof(WaveLds) * L->waves;
    return HS_OK;
}

// Workgroups of `fn` resident per compute unit at `lds` bytes of LDS.
int resident_wgs(const void* fn, int threads, size_t lds, int* per_cu) {
    *per_cu = 0;
    int rc = set_lds_limit(fn, lds);
    if (rc) return rc;
    if (int rc_o = occupancy(fn, threads, lds, per_cu)) return rc_o;
    return HS_OK;
}

// Whether the high-ILP letter loop (more registers per lane) keeps as many
// workgroups resident as the default loop at this LDS footprint: true when
// LDS, not registers, bounds residency (long queries), where the extra reads
// in flight are free.
int prefer_ilp(const void* fn_default, const void* fn_ilp, int threads, size_t lds, bool* ilp) {
    int a = 0, b = 0;
    int rc = resident_wgs(fn_default, threads, lds, &a);
    if (!rc) rc = resident_wgs(fn_ilp, threads, lds, &b);
    if (rc) return rc;
    *ilp = b >= a && b > 0;
    return HS_OK;
}

// Target letters a wavefront of the one-query search keeps in flight: 64
// pairs of targets up to 384 letters, one pair of a target over 12,288.
constexpr int64_t kLettersInFlight = 64 * 384;
constexpr uint32_t kTailGrab = 32;       // counter grabs of the short tail (striped schedule)

template <int kCopies, bool kCount, bool kIlp, int kBits = 8>
int launch_sched(const hs_db* db, const uint8_t* d_q, int32_t qlen, const KParams& kp,
                 const KMatrix& km, int32_t bias, hipStream_t st, const QueryWs& w,
                 int32_t* d_scores, int32_t* d_rounds, uint64_t* d_cells, int32_t* d_max,
                 const QueryLayout& L) {
    const void* fn = (const void*)k_score_sched<kCopies, kCount, kIlp, kBits>;
    const int threads = L.waves * kLanes;
    int rc = set_lds_limit(fn, L.lds);
    if (rc) return rc;
    int per_cu = 0;
    if (int rc_o = occupancy(fn, threads, L.lds, &per_cu)) return rc_o;
    if (per_cu < 1) return fail(HS_ENOMEM, "scoring kernel does not fit on a compute unit");
    // Spread the pairs over every wavefront that can be resident: cap pairs
    // in flight per wavefront, taken cap at a time.  The cap is the smallest
    // of 64, the share that puts every pair in flight at once, and the share
    // that keeps about kLettersInFlight target letters (median length) in
    // flight: one pair of a long target already fills the wavefront's lanes
    // with blocks, and pairs left in the queue balance the wavefronts' loads
    // (32 queries of 2,000-5,000 letters against targets of median 17,000
    // letters ran 1.9 times faster at cap 1 than with every pair in flight).
    const int64_t slots = (int64_t)per_cu * device_cus() * L.waves;
    const int64_t by_len = std::max<int64_t>(1, kLettersInFlight / std::max<int32_t>(db->median_len, 1));
    const int32_t cap = (int32_t)std::min<int64_t>(
        std::min<int64_t>(kLanes, by_len), std::max<int64_t>(1, (db->n_targets + slots - 1) / slots));
    const int64_t want = (db->n_targets + (int64_t)cap * L.waves - 1) / ((int64_t)cap * L.waves);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)per_cu * device_cus(), want));
    // With every lane holding a pair (many short targets), the longest three
    // quarters of the length ranks are striped over the wavefronts and the
    // rest taken from the counter 32 at a time: grabs of 64 positions left
    // the last wavefronts holding up to 64 pairs while others sat idle, and
    // the counter's tail lets the faster wavefronts (older ones take issue
    // priority on a SIMD) take more of the short pairs.  Scoring of the full
    // search: 0.606 ms with grabs of 64, 0.568 ms striping every rank, 0.52 ms
    // with this.
    const uint32_t stride = cap == kLanes ? (uint32_t)grid * (uint32_t)L.waves : 0u;
    const uint32_t r0 = stride ? (uint32_t)(db->n_queue * 3 / 4 / stride) * stride : 0u;
    const uint32_t grab = stride ? kTailGrab : (uint32_t)cap;
    hipLaunchKernelGGL((k_score_sched<kCopies, kCount, kIlp, kBits>), dim3(grid), dim3(threads), L.lds, st,
                       (const PairRec*)db->d_recs, (int32_t)db->n_queue,
                       kBits == 5 ? db->d_letters5 : db->d_letters, d_q, qlen,
                       kp, km, bias, cap, grab, stride, r0, (const uint64_t*)w.draws, w.queue, d_scores,
                       d_rounds,
                       (unsigned long long*)d_cells, d_max);
    HIP_TRY(hipGetLastError());
    return HS_OK;
}

// With `reset`, the draw kernel also sets up the ranking state of the search
// (which then needs no reset launch of its own).
int launch_score(const hs_db* db, const uint8_t* d_q, int32_t qlen, const hs_params* p,
                 hipStream_t st, const QueryWs& w, int32_t* d_scores, int32_t* d_rounds,
                 uint64_t* d_cells, int32_t* d_max, bool reset = false) {
    if (db->n_targets == 0) return HS_OK;
    const KParams kp = kparams(p);
    const KMatrix km = kmatrix(p);
    const int32_t bias = matrix_bias(km);
    const int32_t nq = (int32_t)db->n_queue;
    hipLaunchKernelGGL(k_draws, dim3((2 * (int64_t)nq + 255) / 256), dim3(256), 0, st,
                       (const PairRec*)db->d_recs, nq, kp.seed, w.draws, w.queue, w.tw(),
                       p->min_score, reset ? 1 : 0);
    HIP_TRY(hipGetLastError());
    QueryLayout L;
    int rc = query_layout(qlen, &L);
    if (rc) return rc;
    const bool four = L.copies == 4;
    bool ilp = false;
    rc = four ? prefer_ilp((const void*)k_score_sched<4, false, false>,
                           (const void*)k_score_sched<4, false, true>, L.waves * kLanes, L.lds, &ilp)
              : prefer_ilp((const void*)k_score_sched<1, false, false>,
                           (const void*)k_score_sched<1, false, true>, L.waves * kLanes, L.lds, &ilp);
    if (rc) return rc;
#define HS_SCHED(C, K, I, cells) \
    launch_sched<C, K, I>(db, d_q, qlen, kp, km, bias, st, w, d_scores, d_rounds, cells, d_max, L)
    // the 5-bit image serves launches with four profile copies; the one-copy
    // launch of the longest queries reads the byte image
    if (db->letter_bits == 5 && four) {
        if (d_cells)
            return ilp ? launch_sched<4, true, true, 5>(db, d_q, qlen, kp, km, bias, st, w, d_scores,
                                                        d_rounds, d_cells, d_max, L)
                       : launch_sched<4, true, false, 5>(db, d_q, qlen, kp, km, bias, st, w, d_scores,
                                                         d_rounds, d_cells, d_max, L);
        return ilp ? launch_sched<4, false, true, 5>(db, d_q, qlen, kp, km, bias, st, w, d_scores,
                                                     d_rounds, nullptr, d_max, L)
                   : launch_sched<4, false, false, 5>(db, d_q, qlen, kp, km, bias, st, w, d_scores,
                                                      d_rounds, nullptr, d_max, L);
    }
    if (d_cells) {
        if (four) return ilp ? HS_SCHED(4, true, true, d_cells) : HS_SCHED(4, true, false, d_cells);
        return ilp ? HS_SCHED(1, true, true, d_cells) : HS_SCHED(1, true, false, d_cells);
    }
    if (four) return ilp ? HS_SCHED(4, false, true, nullptr) : HS_SCHED(4, false, false, nullptr);
    return ilp ? HS_SCHED(1, false, true, nullptr) : HS_SCHED(1, false, false, nullptr);
#undef HS_SCHED
}

// Ranking of nq score arrays (query q's scores at scores + q * stride); the
// threshold of each query is in its TopkState.
int launch_rank(const hs_db* db, hipStream_t st, const int32_t* scores, const int32_t* rounds,
                int64_t stride, int32_t nq, int32_t k, const TopkWs& tw, DevHit* d_hits,
                int32_t* d_n_hits) {
    const int32_t n = (int32_t)db->n_targets;
    // about 128 workgroups over all queries (each merges its histogram into
    // the query's with one global atomic per non-empty bin, so fewer, fuller
    // workgroups contend less), at least 1024 scores each
    const int tb = std::max(1, std::min(std::max(1, 128 / nq), (n + 1023) / 1024));
    hipLaunchKernelGGL(k_topk_hist, dim3(tb, nq), dim3(256), 0, st, scores, stride, n, tw);
    hipLaunchKernelGGL(k_topk_pick, dim3(1, nq), dim3(256), 0, st, k, n, tw);
    hipLaunchKernelGGL(k_topk_collect, dim3(tb, nq), dim3(256), 0, st, scores, stride, n, tw);
    const size_t lds = sizeof(uint64_t) * (kSortCap + 8);
    int rc = set_lds_limit((const void*)k_topk_final, lds);
    if (rc) return rc;
    // enough workgroups for k keys and some ties; more keys are strided
    const int fg = std::max(1, std::min(kFinalGroups, (k + kFinalThreads - 1) / kFinalThreads + 1));
    hipLaunchKernelGGL(k_topk_final, dim3(fg, nq), dim3(kFinalThreads), lds, st, scores, stride,
                       rounds, n, k, tw, d_hits, d_n_hits);
    HIP_TRY(hipGetLastError());
    return HS_OK;
}

// Alignments of one query's first n_aln hits: one hit per wavefront, so that
// every alignment is recovered at once.
template <int kCopies>
int launch_trace(const hs_db* db, const uint8_t* d_q, int32_t qlen, const KParams& kp,
                 const KMatrix& km, hipStream_t st, const DevHit* d_hits, const int32_t* d_n_hits,
                 int32_t n_aln, DevAln* d_alns, uint32_t* d_ops, int64_t ops_stride,
                 const QueryLayout& L) {
    const int32_t per_wg = L.waves;
    // a target buffer per wavefront when the LDS allows it (not beside the
    // longest queries' profiles)
    const int32_t pb = profile_region_bytes(qlen, kCopies);
    const bool staged = (size_t)trace_lds_bytes(pb, L.waves) + 16 <= device_lds_limit();
    const size_t lds = staged ? (size_t)trace_lds_bytes(pb, L.waves) : (size_t)trace_stage_offset(pb);
    int rc = set_lds_limit((const void*)k_trace_sched<kCopies>, lds);
    if (rc) return rc;
    hipLaunchKernelGGL((k_trace_sched<kCopies>), dim3((n_aln + per_wg - 1) / per_wg),
                       dim3(L.waves * kLanes), lds, st, db->view(), d_q, qlen, kp, km,
                       matrix_bias(km), d_hits, d_n_hits, n_aln, per_wg, d_alns, d_ops, ops_stride,
                       staged ? (int32_t)sizeof(WaveLds) : 0);
    HIP_TRY(hipGetLastError());
    return HS_OK;
}

// Queues one search.  All pointers are device pointers.
int launch_search(const hs_db* db, const uint8_t* d_q, int32_t qlen, const hs_params* p, int32_t k,
                  int32_t n_aln, hipStream_t st, void* d_ws, DevHit* d_hits, int32_t* d_n_hits,
                  DevAln* d_alns, uint32_t* d_ops, int64_t ops_stride) {
    QueryWs w = carve(d_ws, db->n_targets, db->n_queue);
    if (db->n_targets == 0)   // no draw kernel runs: reset the ranking state here
        hipLaunchKernelGGL(k_topk_reset, dim3(1, 1), dim3(256), 0, st, w.tw(), p->min_score,
                           (const BatchQuery*)nullptr, (uint32_t*)nullptr);
    int rc = launch_score(db, d_q, qlen, p, st, w, w.scores, w.rounds, nullptr, &w.topk->max_score,
                          true);
    if (rc) return rc;
    rc = launch_rank(db, st, w.scores, w.rounds, 0, 1, k, w.tw(), d_hits, d_n_hits);
    if (rc) return rc;
    if (n_aln > 0) {
        const KParams kp = kparams(p);
        const KMatrix km = kmatrix(p);
        QueryLayout L;
        if ((rc = query_layout(qlen, &L))) return rc;
        rc = L.copies == 4
                 ? launch_trace<4>(db, d_q, qlen, kp, km, st, d_hits, d_n_hits, n_aln, d_alns, d_ops,
                                   ops_stride, L)
                 : launch_trace<1>(db, d_q, qlen, kp, km, st, d_hits, d_n_hits, n_aln, d_alns, d_ops,
                                   ops_stride, L);
        if (rc) return rc;
    }
    return HS_OK;
}

// Threshold workspace: the search's own workspace, then the radix sort's
// state, histogram and two key buffers.
size_t threshold_ws_bytes(const hs_db* db) {
    const size_t n = (size_t)std::max<int64_t>(db->n_targets, 1);
    const size_t tiles = (size_t)std::max<int64_t>(rs_tiles(db->n_targets), 1);
    return query_ws_bytes(db->n_targets, db->n_queue, 1) + align_up(sizeof(RsState)) +
           align_up(sizeof(uint32_t) * kRsBins * tiles) +
           align_up(sizeof(uint32_t) * (size_t)rs_segments((int64_t)tiles)) +
           4 * align_up(sizeof(uint32_t) * n);
}

RsWs carve_rs(void* ws, const hs_db* db) {
    const size_t n = (size_t)std::max<int64_t>(db->n_targets, 1);
    const size_t tiles = (size_t)std::max<int64_t>(rs_tiles(db->n_targets), 1);
    char* p = (char*)ws + query_ws_bytes(db->n_targets, db->n_queue, 1);
    RsWs r;
    r.st = (RsState*)p;
    p += align_up(sizeof(RsState));
    r.hist = (uint32_t*)p;
    p += align_up(sizeof(uint32_t) * kRsBins * tiles);
    r.part = (uint32_t*)p;
    p += align_up(sizeof(uint32_t) * (size_t)rs_segments((int64_t)tiles));
    r.v[0] = (uint32_t*)p;
    p += align_up(sizeof(uint32_t) * n);
    r.v[1] = (uint32_t*)p;
    p += align_up(sizeof(uint32_t) * n);
    r.id[0] = (int32_t*)p;
    p += align_up(sizeof(uint32_t) * n);
    r.id[1] = (int32_t*)p;
    return r;
}

// Queues a threshold search: scoring, the radix passes, the ranked hits
// and the alignments of the first n_aln ranks.  All pointers are device
// pointers.
int launch_threshold(const hs_db* db, const uint8_t* d_q, int32_t qlen, const hs_params* p,
                     int64_t cap, int32_t n_aln, hipStream_t st, void* d_ws, DevHit* d_hits,
                     int64_t* d_n, DevAln* d_alns, uint32_t* d_ops, int64_t ops_stride) {
    QueryWs w = carve(d_ws, db->n_targets, db->n_queue);
    RsWs r = carve_rs(d_ws, db);
    hipLaunchKernelGGL(k_rs_reset, dim3(1), dim3(64), 0, st, r.st);
    if (db->n_targets == 0)   // no draw kernel runs: reset the ranking state here
        hipLaunchKernelGGL(k_topk_reset, dim3(1, 1), dim3(256), 0, st, w.tw(), p->min_score,
                           (const BatchQuery*)nullptr, (uint32_t*)nullptr);
    int rc = launch_score(db, d_q, qlen, p, st, w, w.scores, w.rounds, nullptr, &w.topk->max_score,
                          true);
    if (rc) return rc;
    const int32_t n = (int32_t)db->n_targets;
    const int32_t tiles = (int32_t)std::max<int64_t>(rs_tiles(n), 1);
    for (int pass = 0; pass < 4; ++pass) {
        hipLaunchKernelGGL(k_rs_hist, dim3(tiles), dim3(kRsThreads), 0, st, pass,
                           (const int32_t*)w.scores, n, (const TopkState*)w.topk, r, tiles);
        const int64_t L = (int64_t)kRsBins * tiles, G = rs_segments(tiles);
        hipLaunchKernelGGL(k_rs_scan_reduce, dim3((unsigned)G), dim3(kRsThreads), 0, st, pass, r, L);
        hipLaunchKernelGGL(k_rs_scan_top, dim3(1), dim3(kRsScanThreads), 0, st, pass, r, G);
        hipLaunchKernelGGL(k_rs_scan_down, dim3((unsigned)G), dim3(kRsThreads), 0, st, pass, r, L);
        hipLaunchKernelGGL(k_rs_scatter, dim3(tiles), dim3(kRsThreads), 0, st, pass,
                           (const int32_t*)w.scores, n, (const TopkState*)w.topk, r, tiles);
    }
    const int64_t out_blocks = std::max<int64_t>(1, std::min<int64_t>((std::min<int64_t>(cap, n) + 255) / 256, 4096));
    hipLaunchKernelGGL(k_rs_out, dim3((unsigned)out_blocks), dim3(256), 0, st,
                       (const TopkState*)w.topk, r, (const int32_t*)w.rounds, cap, d_hits, d_n);
    HIP_TRY(hipGetLastError());
    if (n_aln > 0) {
        const KParams kp = kparams(p);
        const KMatrix km = kmatrix(p);
        QueryLayout L;
        if ((rc = query_layout(qlen, &L))) return rc;
        rc = L.copies == 4
                 ? launch_trace<4>(db, d_q, qlen, kp, km, st, d_hits, &r.st->n_out, n_aln, d_alns,
                                   d_ops, ops_stride, L)
                 : launch_trace<1>(db, d_q, qlen, kp, km, st, d_hits, &r.st->n_out, n_aln, d_alns,
                                   d_ops, ops_stride, L);
        if (rc) return rc;
    }
    return HS_OK;
}

}  // namespace

// --------------------------------------------------------------------------
// batches: many queries in one persistent scoring launch
// --------------------------------------------------------------------------
struct hs_batch {
    const hs_db* db = nullptr;
    int32_t max_nq = 0, max_qlen = 0, k = 0, n_aln = 0;
    int64_t max_res = 0, ops_stride = 0, max_items = 0, max_titems = 0;
    char* d_mem = nullptr;
    // pinned host mirrors, laid out as the device regions they are copied
    // to or from: the uploads (codes .. alignment items) and the results
    // (hits, hit counts, alignments; packing offsets after them)
    char* h_up = nullptr;
    char* h_down = nullptr;
    const char* d_up_view = nullptr;   // device addresses of h_up and h_down (copied by
    char* d_down_view = nullptr;       // k_copy_segs)
    uint8_t* h_qcodes = nullptr;
    BatchQuery* h_qs = nullptr;
    KMatrix* h_mats = nullptr;
    BatchItem* h_items = nullptr;
    BatchItem* h_titems = nullptr;
    DevHit* h_hits = nullptr;
    int32_t* h_nh = nullptr;
    DevAln* h_alns = nullptr;
    int64_t* h_pos = nullptr;
    uint32_t* h_packed = nullptr;        // the first ops_prefix bytes of the packed ops
    size_t ops_prefix = 0;
    uint8_t* d_qcodes = nullptr;
    BatchQuery* d_qs = nullptr;
    KMatrix* d_mats = nullptr;
    BatchItem* d_items = nullptr;
    BatchItem* d_titems = nullptr;      // alignment work items
    uint32_t* d_ctr = nullptr;          // [0]: scoring items, [1]: alignment items
    int32_t* d_scores = nullptr;        // [max_nq][n_targets]
    int32_t* d_rounds = nullptr;
    uint64_t* d_draws = nullptr;        // round-0 draws, 8 words per hand-out position
    TopkState* d_st = nullptr;
    uint32_t* d_hist = nullptr;
    uint64_t* d_keys = nullptr;
    DevHit* d_hits = nullptr;           // [max_nq][k]
    int32_t* d_n_hits = nullptr;
    DevAln* d_alns = nullptr;           // [max_nq][n_aln]
    uint32_t* d_ops = nullptr;          // [max_nq * n_aln][ops_stride]
    int64_t* d_pos = nullptr;           // packing offsets, max_nq * n_aln + 1
    uint32_t* d_packed = nullptr;
    // queries of the current batch
    int32_t nq = 0, cur_max_qlen = 0;
    std::vector<int32_t> qlens;
    bool table_valid = false;
    uint64_t table_seed = 0;
    // schedule: profile copies, pairs in flight per wavefront, positions per item
    int32_t copies = 0, cap = 0, chunk = 0;
    int32_t fix_copies = 0, fix_cap = 0, fix_chunk = 0;   // 0: chosen automatically
    bool ilp = false;                   // high-ILP letter loop (see prefer_ilp)
    int32_t grid = 0, n_items = 0;
    int32_t waves = kWaves;             // wavefronts per workgroup (LDS permitting)
    int32_t rec = 0;                    // the scoring kernel's record kind (see choose_schedule)
    int32_t swaves = kWaves;            // the scoring kernel's wavefronts per workgroup
    // alignment pass: hits per work item, in flight per wavefront, workgroups
    int32_t tchunk = 0, tcap = 0, tgrid = 0, n_titems = 0;
    bool trace_one = false;          // alignments one hit per wavefront
    bool score_one = false;          // scoring one pair per wavefront
    // graph of one whole search
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec = nullptr;

    TopkWs tw() const {
        TopkWs t;
        t.st = d_st;
        t.hist = d_hist;
        t.keys = d_keys;
        return t;
    }
};

namespace {

constexpr int32_t kMaxChunksPerQuery = 64;

void drop_graph(hs_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
}

void free_batch(hs_batch* b) {
    if (!b) return;
    drop_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    (void)hipFree(b->d_mem);
    if (b->h_up) (void)hipHostFree(b->h_up);
    if (b->h_down) (void)hipHostFree(b->h_down);
    delete b;
}

int64_t round64(int64_t x) { return (x + 63) / 64 * 64; }

// Smallest item size that keeps a query within kMaxChunksPerQuery items.
int32_t min_chunk(const hs_db* db) {
    return (int32_t)std::max<int64_t>(64, round64((db->n_queue + kMaxChunksPerQuery - 1) / kMaxChunksPerQuery));
}

size_t batch_prof_bytes(int32_t qlen, int copies) {
    return align_up((size_t)copies * profile_copy_bytes(profile_stride(qlen)));
}

// Whether `copies` profile copies of queries up to qlen fit in LDS beside at
// least min_waves wavefronts' records.
bool copies_fit(int32_t qlen, int copies, int min_waves = 1) {
    return fit_waves(batch_prof_bytes(qlen, copies)) >= min_waves;
}

}  // namespace

namespace hs_internal {
// LDS class of a query in a batch: 4 when its four profile copies fit beside
// a full workgroup (the launch keeps aligned profile reads), else 1.  A batch
// runs with the class of its longest query.
int batch_lds_class(int32_t qlen) { return copies_fit(qlen, 4, kWaves) ? 4 : 1; }
}  // namespace hs_internal

namespace {

template <int kCopies, bool kCount>
const void* batch_fn(bool ilp) {
    return ilp ? (const void*)k_score_batch<kCopies, kCount, true>
               : (const void*)k_score_batch<kCopies, kCount, false>;
}

const void* batch_kernel(int copies, bool count, bool ilp) {
    if (copies == 4) return count ? batch_fn<4, true>(ilp) : batch_fn<4, false>(ilp);
    return count ? batch_fn<1, true>(ilp) : batch_fn<1, false>(ilp);
}

size_t batch_lds(const hs_batch* b, int copies) {
    return batch_prof_bytes(b->cur_max_qlen, copies) + sizeof(WaveLds) * b->waves;
}
// LDS and kernel of the batch's scoring launch (the wavefront records of
// the long mode are smaller, and its workgroups larger).
size_t rec_bytes(int rec) {
    return rec == 1 ? sizeof(WaveLds16) : rec == 2 ? sizeof(WaveLds64) : sizeof(WaveLds);
}

size_t batch_lds_score(const hs_batch* b, int copies) {
    return b->rec ? batch_prof_bytes(b->cur_max_qlen, copies) + rec_bytes(b->rec) * b->swaves
                  : batch_lds(b, copies);
}

// (the cell-counting kernels of the big workgroups, which run once per
// batch to measure the work, keep the default letter loop: the high-ILP one
// would spill at four wavefronts per SIMD)
template <int kCopies, bool kCount, int kRec>
const void* batch_fn_rec(bool ilp) {
    return ilp && !kCount ? (const void*)k_score_batch<kCopies, kCount, !kCount, kRec>
                          : (const void*)k_score_batch<kCopies, kCount, false, kRec>;
}

template <int kRec>
const void* batch_kernel_rec(int copies, bool count, bool ilp) {
    if (copies == 4) return count ? batch_fn_rec<4, true, kRec>(ilp) : batch_fn_rec<4, false, kRec>(ilp);
    return count ? batch_fn_rec<1, true, kRec>(ilp) : batch_fn_rec<1, false, kRec>(ilp);
}

const void* batch_kernel_score(const hs_batch* b, bool count) {
    if (b->rec == 1) return batch_kernel_rec<1>(b->copies, count, b->ilp);
    if (b->rec == 2) return batch_kernel_rec<2>(b->copies, count, b->ilp);
    return batch_kernel(b->copies, count, b->ilp);
}

// Wavefronts (at most max_w) whose records of `rec_b` bytes fit in one
// workgroup's LDS beside a profile of prof_bytes, and the wavefronts per
// compute unit that gives (workgroups as many as the LDS holds).
int fit_waves_rec(size_t prof_bytes, size_t rec_b, int max_w, int* per_cu_waves) {
    const size_t lim = device_lds_limit();
    for (int w = max_w; w >= 1; --w) {
        const size_t wg = prof_bytes + rec_b * w + 16;
        if (wg <= lim) {
            const int wgs = (int)std::min<size_t>(lim / wg, (size_t)(kBigWaves / w));
            *per_cu_waves = w * std::max(wgs, 1);
            return w;
        }
    }
    *per_cu_waves = 0;
    return 0;
}

// Work items for the current queries: longest queries first, each cut into
// ranges of `chunk` hand-out positions.
// Queues a copy of up to three segments (byte offsets, lengths rounded up
// to 16: every region is 256-byte aligned and padded).
int copy_segments(const void* src, void* dst, hipStream_t st, const int64_t* soff,
                  const int64_t* doff, const int64_t* len, int n) {
    CopySegs sg;
    sg.n = 0;
    int64_t most = 0;
    for (int i = 0; i < n; ++i) {
        if (len[i] <= 0) continue;
        sg.soff[sg.n] = soff[i];
        sg.doff[sg.n] = doff[i];
        sg.len[sg.n] = (len[i] + 15) & ~(int64_t)15;
        most = std::max(most, sg.len[sg.n]);
        ++sg.n;
    }
    if (sg.n == 0) return HS_OK;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((most / 16 + 255) / 256, 256));
    hipLaunchKernelGGL(k_copy_segs, dim3((unsigned)blocks), dim3(256), 0, st, (const uint4*)src,
                       (uint4*)dst, sg);
    HIP_TRY(hipGetLastError());
    return HS_OK;
}

// Upload of mirror segments to the same offsets of the device region.
int pull_segments(hs_batch* b, hipStream_t st, const int64_t* off, const int64_t* len, int n) {
    return copy_segments(b->d_up_view, b->d_mem, st, off, off, len, n);
}

int upload_items(hs_batch* b, hipStream_t st) {
    std::vector<int32_t> order((size_t)b->nq);
    for (int32_t q = 0; q < b->nq; ++q) order[(size_t)q] = q;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return b->qlens[(size_t)x] > b->qlens[(size_t)y]; });
    std::vector<BatchItem> items;
    const int64_t nqueue = b->db->n_queue;
    for (int32_t q : order)
        for (int64_t lo = 0; lo < nqueue; lo += b->chunk) {
            BatchItem it;
            it.q = q;
            it.lo = (uint32_t)lo;
            it.hi = (uint32_t)std::min<int64_t>(lo + b->chunk, nqueue);
            it.pad_ = 0;
            items.push_back(it);
        }
    if ((int64_t)items.size() > b->max_items) return fail(HS_EINVAL, "too many work items");
    b->n_items = (int32_t)items.size();
    // alignment items: each query's first n_aln ranks, in ranges of tchunk.
    // A small batch, whose items of one hit per wavefront all fit on the
    // device at once, replays one hit per wavefront; a large one keeps each
    // query's hits in one item, several per wavefront (slot-based).
    std::vector<BatchItem> titems;
    const int64_t one_items = (int64_t)b->nq * ((b->n_aln + b->waves - 1) / b->waves);
    b->trace_one = b->n_aln > 0 && one_items <= std::min<int64_t>(b->max_titems, 2 * (int64_t)device_cus());
    b->tchunk = b->trace_one ? b->waves : std::max(b->n_aln, 1);
    b->tcap = std::min(kLanes, (b->tchunk + b->waves - 1) / b->waves);
    for (int32_t q : order)
        for (int32_t lo = 0; lo < b->n_aln; lo += b->tchunk) {
            BatchItem it;
            it.q = q;
            it.lo = (uint32_t)lo;
            it.hi = (uint32_t)std::min(lo + b->tchunk, b->n_aln);
            it.pad_ = 0;
            titems.push_back(it);
        }
    if ((int64_t)titems.size() > b->max_titems) return fail(HS_EINVAL, "too many alignment items");
    b->n_titems = (int32_t)titems.size();
    // both item lists in one copy from the pinned mirror (their device
    // regions lie back to back), then wait for every upload of the batch
    if (!items.empty()) std::memcpy(b->h_items, items.data(), items.size() * sizeof(BatchItem));
    if (!titems.empty()) std::memcpy(b->h_titems, titems.data(), titems.size() * sizeof(BatchItem));
    const int64_t off[2] = {(const char*)b->h_items - b->h_up, (const char*)b->h_titems - b->h_up};
    const int64_t len[2] = {(int64_t)(items.size() * sizeof(BatchItem)),
                            (int64_t)(titems.size() * sizeof(BatchItem))};
    if (int rc = pull_segments(b, st, off, len, 2)) return rc;
    HIP_TRY(hipStreamSynchronize(st));
    const void* fn = batch_kernel_score(b, false);
    const size_t lds = batch_lds_score(b, b->copies);
    const int threads = b->swaves * kLanes;
    int rc = set_lds_limit(fn, lds);
    if (!rc) rc = set_lds_limit(batch_kernel_score(b, true), lds);
    if (!rc && b->score_one) {
        const bool four = b->copies == 4;
        rc = set_lds_limit(four ? (const void*)k_score_one<4, false> : (const void*)k_score_one<1, false>, lds);
        if (!rc) rc = set_lds_limit(four ? (const void*)k_score_one<4, true> : (const void*)k_score_one<1, true>, lds);
    }
    if (rc) return rc;
    int per_cu = 0;
    if (int rc_o = occupancy(fn, threads, lds, &per_cu)) return rc_o;
    if (per_cu < 1) return fail(HS_ENOMEM, "batch scoring kernel does not fit on a compute unit");
    b->grid = (int32_t)std::max<int64_t>(1, std::min<int64_t>((int64_t)per_cu * device_cus(), b->n_items));
    const void* tfn = b->copies == 4 ? (const void*)k_trace_batch<4> : (const void*)k_trace_batch<1>;
    if ((rc = set_lds_limit(tfn, batch_lds(b, b->copies)))) return rc;
    per_cu = 0;
    if (int rc_o = occupancy(tfn, b->waves * kLanes, batch_lds(b, b->copies), &per_cu)) return rc_o;
    if (per_cu < 1) return fail(HS_ENOMEM, "batch alignment kernel does not fit on a compute unit");
    b->tgrid = (int32_t)std::max<int64_t>(1, std::min<int64_t>((int64_t)per_cu * device_cus(), b->n_titems));
    drop_graph(b);
    return HS_OK;
}

// Picks the schedule fields not fixed by the caller: four profile copies when
// they fit, 64 pairs in flight per wavefront, and items small enough that
// every workgroup gets about four.
int choose_schedule(hs_batch* b, hipStream_t st) {
    b->copies = b->fix_copies ? b->fix_copies : (copies_fit(b->cur_max_qlen, 4, kWaves) ? 4 : 1);
    if (!copies_fit(b->cur_max_qlen, b->copies))
        return fail(HS_EINVAL, "profile copies do not fit in LDS for the longest query");
    b->waves = fit_waves(batch_prof_bytes(b->cur_max_qlen, b->copies));
    b->rec = 0;
    b->swaves = b->waves;
    b->cap = b->fix_cap ? b->fix_cap : kLanes;
    int rc = prefer_ilp(batch_kernel(b->copies, false, false), batch_kernel(b->copies, false, true),
                        b->waves * kLanes, batch_lds(b, b->copies), &b->ilp);
    if (rc) return rc;
    int per_cu = 0;
    {
        const void* fn = batch_kernel(b->copies, false, b->ilp);
        const size_t lds = batch_lds(b, b->copies);
        rc = set_lds_limit(fn, lds);
        if (rc) return rc;
        if (int rc_o = occupancy(fn, b->waves * kLanes, lds, &per_cu)) return rc_o;
    }
    const int64_t wgs = (int64_t)std::max(per_cu, 1) * device_cus();
    // A batch whose items of one pair per wavefront all fit on the device at
    // once is scored one pair per wavefront, all lanes on the pair: the
    // chains of steps, not the lanes, set its time.
    const int64_t one_items = (int64_t)b->nq * ((b->db->n_queue + b->waves - 1) / b->waves);
    b->score_one = !b->fix_cap && !b->fix_chunk && b->db->n_queue > 0 &&
                   one_items <= std::min<int64_t>(wgs, b->max_items);
    if (b->score_one) {
        b->chunk = b->waves;
        b->cap = 1;
        return upload_items(b, st);
    }
    if (b->fix_chunk) {
        b->chunk = std::max(b->fix_chunk, min_chunk(b->db));
    } else {
        const int64_t want = (int64_t)b->nq * b->db->n_queue / (4 * wgs);
        b->chunk = (int32_t)std::min<int64_t>(round64(std::max<int64_t>(b->db->n_queue, 64)),
                                              std::max<int64_t>(round64(want), min_chunk(b->db)));
    }
    // pairs in flight per wavefront: an item's positions shared by all the
    // workgroup's wavefronts (with 64, the first wavefront would take a
    // small item whole and leave the others idle), and no more than keep
    // about kLettersInFlight target letters in flight (median length), as in
    // the one-query kernel: on long targets the queue then still holds pairs
    // that balance the wavefronts (32 queries of 2,000-5,000 letters against
    // targets of median 17,000 letters took 169 ms at 32 pairs in flight)
    if (!b->fix_cap) {
        const int32_t by_len = (int32_t)std::max<int64_t>(
            1, kLettersInFlight / std::max<int32_t>(b->db->median_len, 1));
        b->cap = std::min(std::min(kLanes, by_len), std::max(1, (b->chunk + b->waves - 1) / b->waves));
    }
    // Record kind: the smaller records (16 slots when at most 16 pairs are
    // in flight, else 64) in workgroups of up to 16 wavefronts when they put
    // more wavefronts on a compute unit than the full records: the
    // long-sequence batch (a 121 KB profile) gets 16 instead of 8 (93 ms ->
    // 77 ms, with 4 pairs in flight), the 256-query batch with four copies
    // (104 KB) 15 instead of 8 (0.90 ms -> 0.85 ms).
    {
        const size_t prof = batch_prof_bytes(b->cur_max_qlen, b->copies);
        int best = 0;
        fit_waves_rec(prof, sizeof(WaveLds), kWaves, &best);
        for (int rec = 1; rec <= 2; ++rec) {
            if (b->cap > rec_slots(rec)) continue;
            int cu = 0;
            const int w = fit_waves_rec(prof, rec_bytes(rec), kBigWaves, &cu);
            if (cu > best) {
                best = cu;
                b->rec = rec;
                b->swaves = w;
            }
        }
    }
    return upload_items(b, st);
}

// The scoring launch of a batch with the smaller records (kind kRec).
template <int kCopies, bool kCount, bool kIlp, int kRec>
void launch_batch_rec(const hs_batch* b, hipStream_t st, uint64_t* d_cells) {
    const hs_db* db = b->db;
    hipLaunchKernelGGL((k_score_batch<kCopies, kCount, kIlp, kRec>), dim3(b->grid), dim3(b->swaves * kLanes),
                       batch_lds_score(b, kCopies), st, (const BatchQuery*)b->d_qs,
                       (const KMatrix*)b->d_mats, (const uint8_t*)b->d_qcodes,
                       (const BatchItem*)b->d_items, b->n_items, b->d_ctr,
                       (int32_t)batch_prof_bytes(b->cur_max_qlen, kCopies), b->cap,
                       (const PairRec*)db->d_recs, (const uint8_t*)db->d_letters,
                       (const uint64_t*)b->d_draws, b->d_scores, b->d_rounds,
                       (int64_t)db->n_targets, &b->d_st->max_score,
                       (int32_t)(sizeof(TopkState) / sizeof(int32_t)), (unsigned long long*)d_cells);
}

template <int kCopies, bool kCount, bool kIlp>
void launch_batch_kernel(const hs_batch* b, hipStream_t st, uint64_t* d_cells) {
    const hs_db* db = b->db;
    if (b->score_one) {
        hipLaunchKernelGGL((k_score_one<kCopies, kCount>), dim3(b->grid), dim3(b->waves * kLanes),
                           batch_lds(b, kCopies), st, (const BatchQuery*)b->d_qs,
                           (const KMatrix*)b->d_mats, (const uint8_t*)b->d_qcodes,
                           (const BatchItem*)b->d_items, b->n_items, b->d_ctr,
                           (int32_t)batch_prof_bytes(b->cur_max_qlen, kCopies),
                           (const PairRec*)db->d_recs, (const uint8_t*)db->d_letters,
                           (const uint64_t*)b->d_draws, b->d_scores, b->d_rounds,
                           (int64_t)db->n_targets, &b->d_st->max_score,
                           (int32_t)(sizeof(TopkState) / sizeof(int32_t)), (unsigned long long*)d_cells);
        return;
    }
    if (b->rec == 1) {
        launch_batch_rec<kCopies, kCount, kIlp && !kCount, 1>(b, st, d_cells);
        return;
    }
    if (b->rec == 2) {
        launch_batch_rec<kCopies, kCount, kIlp && !kCount, 2>(b, st, d_cells);
        return;
    }
    hipLaunchKernelGGL((k_score_batch<kCopies, kCount, kIlp>), dim3(b->grid), dim3(b->waves * kLanes),
                       batch_lds(b, kCopies), st, (const BatchQuery*)b->d_qs,
                       (const KMatrix*)b->d_mats, (const uint8_t*)b->d_qcodes,
                       (const BatchItem*)b->d_items, b->n_items, b->d_ctr,
                       (int32_t)batch_prof_bytes(b->cur_max_qlen, kCopies), b->cap,
                       (const PairRec*)db->d_recs, (const uint8_t*)db->d_letters,
                       (const uint64_t*)b->d_draws, b->d_scores, b->d_rounds,
                       (int64_t)db->n_targets, &b->d_st->max_score,
                       (int32_t)(sizeof(TopkState) / sizeof(int32_t)), (unsigned long long*)d_cells);
}

// Scoring of the current batch: state reset, then the persistent kernel.
int enqueue_batch_score(const hs_batch* b, hipStream_t st, uint64_t* d_cells) {
    hipLaunchKernelGGL(k_topk_reset, dim3(8, b->nq), dim3(256), 0, st, b->tw(), 0,
                       (const BatchQuery*)b->d_qs, b->d_ctr);
    HIP_TRY(hipGetLastError());
    if (b->db->n_targets == 0 || b->n_items == 0) return HS_OK;
    const bool c = d_cells != nullptr;
    if (b->copies == 4) {
        if (b->ilp) c ? launch_batch_kernel<4, true, true>(b, st, d_cells)
                      : launch_batch_kernel<4, false, true>(b, st, nullptr);
        else c ? launch_batch_kernel<4, true, false>(b, st, d_cells)
               : launch_batch_kernel<4, false, false>(b, st, nullptr);
    } else {
        if (b->ilp) c ? launch_batch_kernel<1, true, true>(b, st, d_cells)
                      : launch_batch_kernel<1, false, true>(b, st, nullptr);
        else c ? launch_batch_kernel<1, true, false>(b, st, d_cells)
               : launch_batch_kernel<1, false, false>(b, st, nullptr);
    }
    HIP_TRY(hipGetLastError());
    return HS_OK;
}

template <int kCopies>
void launch_trace_batch(const hs_batch* b, hipStream_t st) {
    hipLaunchKernelGGL((k_trace_batch<kCopies>), dim3(b->tgrid), dim3(b->waves * kLanes),
                       batch_lds(b, kCopies), st, b->db->view(), (const BatchQuery*)b->d_qs,
                       (const KMatrix*)b->d_mats, (const uint8_t*)b->d_qcodes,
                       (const BatchItem*)b->d_titems, b->n_titems, b->d_ctr + 1,
                       (int32_t)batch_prof_bytes(b->cur_max_qlen, kCopies), b->tcap,
                       (int32_t)b->trace_one, b->k,
                       (const DevHit*)b->d_hits, (const int32_t*)b->d_n_hits, b->n_aln,
                       b->d_alns, b->d_ops, b->ops_stride);
}

// The whole search of the current batch: scoring, ranking, alignments.
// Kernel launches only (no allocation, copy or fill), so it can be captured.
int enqueue_batch(const hs_batch* b, hipStream_t st) {
    int rc = enqueue_batch_score(b, st, nullptr);
    if (rc) return rc;
    rc = launch_rank(b->db, st, b->d_scores, b->d_rounds, b->db->n_targets, b->nq, b->k, b->tw(),
                     b->d_hits, b->d_n_hits);
    if (rc) return rc;
    if (b->n_aln > 0 && b->n_titems > 0) {
        if (b->copies == 4) launch_trace_batch<4>(b, st);
        else launch_trace_batch<1>(b, st);
        HIP_TRY(hipGetLastError());
    }
    return HS_OK;
}

int check_batch_ready(const hs_batch* b) {
    if (!b) return fail(HS_EINVAL, "batch is NULL");
    if (b->nq < 1) return fail(HS_EINVAL, "no queries set on the batch");
    return HS_OK;
}

}  // namespace

// Workspace of hs_search_dev_noalloc: device memory that comes with the code
// object, so that the call allocates nothing.  Each device the library runs
// on holds its own copy until the process ends.  Host code never passes this
// name to a kernel or a copy (on the host it is only a stand-in for the
// symbol): it uses the device address taken below.
static __device__ __align__(256) uint8_t scratch[HS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];   // device address of `scratch`, per device

// Device address of the current device's scratch array, taken once per
// device with that device current.
int scratch_address(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(HS_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(HS_EDEVICE, "no device address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return HS_OK;
}
}  // namespace

// --------------------------------------------------------------------------
// C ABI
// --------------------------------------------------------------------------
extern "C" {

void hs_params_default(hs_params* p) {
    if (!p) return;
    p->gop = 10;
    p->gep = 5;
    p->pgp = 0;
    p->lfactor_q16 = 32768;
    p->sfactor_q16 = 65536;
    p->minfactor_q16 = 32768;
    p->rounds = 1;
    p->min_score = INT32_MIN;
    p->seed = 0;
    p->matrix = nullptr;
}

int hs_params_check(const hs_params* p) { return check_params(p); }

void hs_builtin_matrix(int8_t* out) {
    if (out) std::memcpy(out, kBlosum62, sizeof(kBlosum62));
}

int hs_encode(const char* ascii, int64_t n, uint8_t* codes) {
    if (n < 0 || (n > 0 && (!ascii || !codes))) return fail(HS_EINVAL, "bad arguments to hs_encode");
    // one pass without a branch per letter (invalid letters map to -1, so
    // the OR of all codes is negative exactly when one is); the position of
    // the first bad letter is looked up only then
    int bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int c = kCodes.t[(unsigned char)ascii[i]];
        bad |= c;
        codes[i] = (uint8_t)c;
    }
    if (bad < 0) {
        int64_t i = 0;
        while (kCodes.t[(unsigned char)ascii[i]] >= 0) ++i;
        return fail(HS_EINVAL, "residue outside the alphabet at position " + std::to_string(i));
    }
    return HS_OK;
}

int hs_db_load(const char* residues, const int64_t* offsets, int64_t n_targets, void* stream,
               hs_db** out) {
    if (!out) return fail(HS_EINVAL, "out is NULL");
    if (n_targets < 0 || n_targets > INT32_MAX / 2) return fail(HS_EINVAL, "bad n_targets");
    if (n_targets > 0 && (!offsets || !residues)) return fail(HS_EINVAL, "NULL residues or offsets");
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> len((size_t)n_targets);
    std::vector<int64_t> rel((size_t)n_targets);
    for (int64_t i = 0; i < n_targets; ++i) {
        const int64_t L = offsets[i + 1] - offsets[i];
        if (L < 1 || L > HS_MAX_SEQ)
            return fail(HS_EINVAL, "target " + std::to_string(i) + " has length outside [1, HS_MAX_SEQ]");
        len[(size_t)i] = (int32_t)L;
        rel[(size_t)i] = offsets[i] - offsets[0];
    }
    const int64_t total = n_targets ? offsets[n_targets] - offsets[0] : 0;
    // hand-out order: longest first, ties by index
    std::vector<int32_t> order((size_t)n_targets);
    for (int64_t i = 0; i < n_targets; ++i) order[(size_t)i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return len[(size_t)a] > len[(size_t)b]; });

    hs_db* db = new hs_db();
    db->n_targets = n_targets;
    db->n_residues = total;
    db->median_len = n_targets ? len[(size_t)order[(size_t)(n_targets / 2)]] : 0;
    db->lens_desc.resize((size_t)n_targets);
    for (int64_t i = 0; i < n_targets; ++i) db->lens_desc[(size_t)i] = len[(size_t)order[(size_t)i]];
    int rc = HS_OK;
    int32_t* d_err = nullptr;
    auto cleanup = [&](int code) {
        (void)hipFree(d_err);
        if (code != HS_OK) free_db(db);
        return code;
    };
    // Hand-out order: wavefronts take 64 consecutive positions at a time, so
    // position 64 b + i holds the target of length rank i * nb + b: every
    // batch of 64 gets one target of each length stratum, and the longest
    // targets go out first, one per batch.  Unused positions hold id -1.
    const int64_t nb = (n_targets + kGrabSize - 1) / kGrabSize;
    db->n_queue = nb * kGrabSize;
    std::vector<PairRec> recs((size_t)db->n_queue);
    for (int64_t b = 0; b < nb; ++b)
        for (int64_t i = 0; i < kGrabSize; ++i) {
            const int64_t rank = i * nb + b;
            PairRec& r = recs[(size_t)(b * kGrabSize + i)];
            if (rank < n_targets) {
                const int32_t id = order[(size_t)rank];
                r.id = id;
                r.len = len[(size_t)id];
                r.offset = rel[(size_t)id];
            } else {
                r.id = -1;
                r.len = 0;
                r.offset = 0;
            }
        }
    if ((rc = dev_alloc(&db->d_letters, (size_t)total + kLetterPad, &db->device_bytes)) ||
        (rc = dev_alloc(&db->d_offsets, (size_t)n_targets, &db->device_bytes)) ||
        (rc = dev_alloc(&db->d_lens, (size_t)n_targets, &db->device_bytes)) ||
        (rc = dev_alloc(&db->d_order, (size_t)n_targets, &db->device_bytes)) ||
        (rc = dev_alloc(&db->d_recs, recs.size(), &db->device_bytes)) ||
        (rc = dev_alloc(&d_err, 1, nullptr)))
        return cleanup(rc);
    auto h2d = [&](void* dst, const void* src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
    };
    if (h2d(db->d_letters, residues + (n_targets ? offsets[0] : 0), (size_t)total) != hipSuccess ||
        h2d(db->d_offsets, rel.data(), rel.size() * 8) != hipSuccess ||
        h2d(db->d_lens, len.data(), len.size() * 4) != hipSuccess ||
        h2d(db->d_order, order.data(), order.size() * 4) != hipSuccess ||
        h2d(db->d_recs, recs.data(), recs.size() * sizeof(PairRec)) != hipSuccess ||
        hipMemsetAsync(d_err, 0, sizeof(int32_t), st) != hipSuccess ||
        hipMemsetAsync(db->d_letters + total, kZeroRow, kLetterPad, st) != hipSuccess ||
        hipMemcpyToSymbolAsync(HIP_SYMBOL(c_codes), kCodes.t, 256, 0, hipMemcpyHostToDevice, st) !=
            hipSuccess)
        return cleanup(fail(HS_EDEVICE, "copy to device failed"));
    if (total > 0) {
        const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
        hipLaunchKernelGGL(k_encode, dim3((unsigned)blocks), dim3(256), 0, st, db->d_letters, total,
                           d_err);
        if (hipGetLastError() != hipSuccess) return cleanup(fail(HS_EDEVICE, "encode launch failed"));
    }
    int32_t err = 0;
    if (hipMemcpyAsync(&err, d_err, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return cleanup(fail(HS_EDEVICE, "database upload failed"));
    if (err) return cleanup(fail(HS_EINVAL, "database holds a residue outside the alphabet"));
    *out = db;
    return cleanup(HS_OK);
}

int hs_db_set_letters(hs_db* db, int32_t bits, void* stream) {
    if (!db) return fail(HS_EINVAL, "db is NULL");
    if (bits != 8 && bits != 5) return fail(HS_EINVAL, "bits must be 8 or 5");
    if (bits == 5 && !db->d_letters5) {
        const int64_t n = db->n_residues;
        const int64_t n_words = (5 * (n + kLetterPad) + 31) / 32 + 4;
        uint32_t* d = nullptr;
        if (int rc = dev_alloc(&d, (size_t)n_words, &db->device_bytes)) return rc;
        hipStream_t st = (hipStream_t)stream;
        const int64_t blocks = std::min<int64_t>((n_words + 255) / 256, 65536);
        hipLaunchKernelGGL(k_pack5, dim3((unsigned)blocks), dim3(256), 0, st, db->d_letters, n, n_words, d);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
            (void)hipFree(d);
            return fail(HS_EDEVICE, "packing the 5-bit letter image failed");
        }
        db->d_letters5 = (uint8_t*)d;
    }
    db->letter_bits = bits;
    return HS_OK;
}

int hs_db_free(hs_db* db) {
    free_db(db);
    return HS_OK;
}

int hs_db_info(const hs_db* db, int64_t* n_targets, int64_t* n_residues, int64_t* device_bytes) {
    if (!db) return fail(HS_EINVAL, "db is NULL");
    if (n_targets) *n_targets = db->n_targets;
    if (n_residues) *n_residues = db->n_residues;
    if (device_bytes) *device_bytes = db->device_bytes;
    return HS_OK;
}

size_t hs_workspace_bytes(const hs_db* db, int32_t nq, int32_t max_qlen, int32_t k, int32_t n_aln) {
    (void)max_qlen;
    (void)n_aln;
    if (!db || nq < 1) return 0;
    return (size_t)nq * query_ws_bytes(db->n_targets, db->n_queue, k);
}

int hs_search_dev(const hs_db* db, const uint8_t* d_qcodes, int32_t qlen, const hs_params* params,
                  int32_t k, int32_t n_aln, void* stream, void* d_ws, size_t ws_bytes,
                  hs_hit* d_hits, int32_t* d_n_hits, hs_aln* d_alns, uint32_t* d_ops,
                  int64_t ops_stride) {
    int rc = check_search_args(db, qlen, params, k, n_aln);
    if (rc) return rc;
    if (!d_qcodes || !d_ws || !d_hits || !d_n_hits || (n_aln > 0 && (!d_alns || !d_ops)))
        return fail(HS_EINVAL, "NULL device pointer");
    if (ws_bytes < hs_workspace_bytes(db, 1, qlen, k, n_aln))
        return fail(HS_ENOSPC, "workspace too small");
    if (n_aln > 0 && ops_stride < 2 * (int64_t)qlen + 2) return fail(HS_EINVAL, "ops_stride too small");
    return launch_search(db, d_qcodes, qlen, params, k, n_aln, (hipStream_t)stream, d_ws,
                         (DevHit*)d_hits, d_n_hits, (DevAln*)d_alns, d_ops, ops_stride);
}

int hs_search_dev_noalloc(const hs_db* db, const uint8_t* d_qcodes, int32_t qlen,
                          const hs_params* params, int32_t k, int32_t n_aln, void* stream,
                          hs_hit* d_hits, int32_t* d_n_hits, hs_aln* d_alns, uint32_t* d_ops,
                          int64_t ops_stride) {
    int rc = check_search_args(db, qlen, params, k, n_aln);
    if (rc) return rc;
    if (!d_qcodes || !d_hits || !d_n_hits || (n_aln > 0 && (!d_alns || !d_ops)))
        return fail(HS_EINVAL, "NULL device pointer");
    if (n_aln > 0 && ops_stride < 2 * (int64_t)qlen + 2) return fail(HS_EINVAL, "ops_stride too small");
    const size_t need = hs_workspace_bytes(db, 1, qlen, k, n_aln);
    if (need > (size_t)HS_NOALLOC_SCRATCH_BYTES)
        return fail(HS_ENOMEM, "database needs a workspace of " + std::to_string(need) +
                                   " bytes, above the static scratch of " +
                                   std::to_string((size_t)HS_NOALLOC_SCRATCH_BYTES) +
                                   " (use hs_search_dev with a workspace)");
    void* ws = nullptr;
    if ((rc = scratch_address(&ws))) return rc;
    // every piece of state the search needs zeroed (queue counter, ranking
    // state) is reset by its own kernels, so the previous call's contents do
    // no harm
    return launch_search(db, d_qcodes, qlen, params, k, n_aln, (hipStream_t)stream, ws,
                         (DevHit*)d_hits, d_n_hits, (DevAln*)d_alns, d_ops, ops_stride);
}

int hs_search(const hs_db* db, const char* query, int32_t qlen, const hs_params* params, int32_t k,
              int32_t n_aln, void* stream, hs_hit* hits, int32_t* n_hits, hs_aln* alns,
              int32_t* n_alns, uint32_t* ops, int64_t ops_cap, int64_t* ops_used) {
    int rc = check_search_args(db, qlen, params, k, n_aln);
    if (rc) return rc;
    if (!query || !hits || !n_hits || (n_aln > 0 && (!alns || !n_alns || !ops_used)))
        return fail(HS_EINVAL, "NULL output pointer");
    std::vector<uint8_t> qc((size_t)qlen);
    if ((rc = hs_encode(query, qlen, qc.data()))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t stride = 2 * (int64_t)qlen + 2;
    const size_t ws = hs_workspace_bytes(db, 1, qlen, k, n_aln);
    const size_t o_q = 0, o_hits = align_up((size_t)qlen), o_nh = o_hits + align_up(sizeof(DevHit) * k),
                 o_alns = o_nh + kAlign, o_ops = o_alns + align_up(sizeof(DevAln) * std::max(n_aln, 1)),
                 o_ws = o_ops + align_up(sizeof(uint32_t) * (size_t)stride * std::max(n_aln, 1)),
                 total = o_ws + ws;
    char* d = nullptr;
    if (hipMallocAsync((void**)&d, total, st) != hipSuccess)
        return fail(HS_ENOMEM, "device workspace allocation failed");
    std::vector<DevHit> h_hits((size_t)k);
    std::vector<DevAln> h_alns((size_t)std::max(n_aln, 1));
    std::vector<uint32_t> h_ops((size_t)stride * std::max(n_aln, 1));
    int32_t nh = 0;
    rc = HS_OK;
    if (hipMemcpyAsync(d + o_q, qc.data(), (size_t)qlen, hipMemcpyHostToDevice, st) != hipSuccess)
        rc = fail(HS_EDEVICE, "query copy failed");
    if (!rc)
        rc = launch_search(db, (const uint8_t*)(d + o_q), qlen, params, k, n_aln, st, d + o_ws,
                           (DevHit*)(d + o_hits), (int32_t*)(d + o_nh), (DevAln*)(d + o_alns),
                           (uint32_t*)(d + o_ops), stride);
    if (!rc && (hipMemcpyAsync(h_hits.data(), d + o_hits, sizeof(DevHit) * k, hipMemcpyDeviceToHost, st) ||
                hipMemcpyAsync(&nh, d + o_nh, 4, hipMemcpyDeviceToHost, st) ||
                (n_aln > 0 && hipMemcpyAsync(h_alns.data(), d + o_alns, sizeof(DevAln) * n_aln,
                                             hipMemcpyDeviceToHost, st)) ||
                (n_aln > 0 && hipMemcpyAsync(h_ops.data(), d + o_ops, sizeof(uint32_t) * stride * n_aln,
                                             hipMemcpyDeviceToHost, st)) ||
                hipStreamSynchronize(st)))
        rc = fail(HS_EDEVICE, "search failed on the device");
    (void)hipFreeAsync(d, st);
    if (rc) return rc;
    const int32_t na = std::min(n_aln, nh);
    int64_t need = 0;
    for (int32_t i = 0; i < na; ++i) need += h_alns[(size_t)i].n_ops;
    if (n_aln > 0) {
        *ops_used = need;
        if (need > ops_cap) return fail(HS_ENOSPC, "ops buffer too small");
    }
    std::memcpy(hits, h_hits.data(), sizeof(DevHit) * (size_t)nh);
    *n_hits = nh;
    if (n_aln > 0) {
        int64_t off = 0;
        for (int32_t i = 0; i < na; ++i) {
            const DevAln& a = h_alns[(size_t)i];
            std::memcpy(ops + off, h_ops.data() + a.ops_off, sizeof(uint32_t) * a.n_ops);
            alns[i].target_id = a.target_id;
            alns[i].score = a.score;
            alns[i].n_ops = a.n_ops;
            alns[i].ops_off = off;
            off += a.n_ops;
        }
        *n_alns = na;
    }
    return HS_OK;
}

int hs_score_dev(const hs_db* db, const uint8_t* d_qcodes, int32_t qlen, const hs_params* params,
                 void* stream, void* d_ws, size_t ws_bytes, int32_t* d_scores, int32_t* d_rounds,
                 uint64_t* d_cells) {
    if (!db) return fail(HS_EINVAL, "db is NULL");
    if (qlen < 1 || qlen > HS_MAX_QUERY) return fail(HS_EINVAL, "qlen must lie in [1, HS_MAX_QUERY]");
    int rc = check_params(params);
    if (rc) return rc;
    if (!d_qcodes || !d_scores || !d_ws) return fail(HS_EINVAL, "NULL device pointer");
    if (ws_bytes < hs_workspace_bytes(db, 1, qlen, 1, 0)) return fail(HS_ENOSPC, "workspace too small");
    QueryWs w = carve(d_ws, db->n_targets, db->n_queue);
    return launch_score(db, d_qcodes, qlen, params, (hipStream_t)stream, w, d_scores, d_rounds,
                        d_cells, nullptr);
}

size_t hs_threshold_workspace_bytes(const hs_db* db) {
    if (!db) return 0;
    return threshold_ws_bytes(db);
}

int hs_search_threshold_dev(const hs_db* db, const uint8_t* d_qcodes, int32_t qlen,
                            const hs_params* params, int64_t cap, int32_t n_aln, void* stream,
                            void* d_ws, size_t ws_bytes, hs_hit* d_hits, int64_t* d_n,
                            hs_aln* d_alns, uint32_t* d_ops, int64_t ops_stride) {
    int rc = check_threshold_args(db, qlen, params, cap, n_aln);
    if (rc) return rc;
    if (!d_qcodes || !d_ws || !d_n || (cap > 0 && !d_hits) || (n_aln > 0 && (!d_alns || !d_ops)))
        return fail(HS_EINVAL, "NULL device pointer");
    if (n_aln > cap) return fail(HS_EINVAL, "n_aln must not exceed cap");
    if (ws_bytes < threshold_ws_bytes(db)) return fail(HS_ENOSPC, "workspace too small");
    if (n_aln > 0 && ops_stride < 2 * (int64_t)qlen + 2) return fail(HS_EINVAL, "ops_stride too small");
    return launch_threshold(db, d_qcodes, qlen, params, cap, n_aln, (hipStream_t)stream, d_ws,
                            (DevHit*)d_hits, d_n, (DevAln*)d_alns, d_ops, ops_stride);
}

int hs_search_threshold(const hs_db* db, const char* query, int32_t qlen, const hs_params* params,
                        int64_t cap, int32_t n_aln, void* stream, hs_hit* hits, int64_t* n_hits,
                        hs_aln* alns, int32_t* n_alns, uint32_t* ops, int64_t ops_cap,
                        int64_t* ops_used) {
    int rc = check_threshold_args(db, qlen, params, cap, n_aln);
    if (rc) return rc;
    if (!query || !n_hits || (cap > 0 && !hits) || (n_aln > 0 && (!alns || !n_alns || !ops_used)))
        return fail(HS_EINVAL, "NULL output pointer");
    std::vector<uint8_t> qc((size_t)qlen);
    if ((rc = hs_encode(query, qlen, qc.data()))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t stride = 2 * (int64_t)qlen + 2;
    // the device keeps at most all targets' ranks, whatever the caller's cap
    const int64_t dcap = std::min<int64_t>(cap, db->n_targets);
    const int32_t na = (int32_t)std::min<int64_t>(n_aln, dcap);
    const size_t ws = threshold_ws_bytes(db);
    const size_t o_q = 0, o_n = align_up((size_t)qlen), o_hits = o_n + kAlign,
                 o_alns = o_hits + align_up(sizeof(DevHit) * (size_t)std::max<int64_t>(dcap, 1)),
                 o_ops = o_alns + align_up(sizeof(DevAln) * std::max(na, 1)),
                 o_ws = o_ops + align_up(sizeof(uint32_t) * (size_t)stride * std::max(na, 1)),
                 total = o_ws + ws;
    char* d = nullptr;
    if (hipMallocAsync((void**)&d, total, st) != hipSuccess)
        return fail(HS_ENOMEM, "device workspace allocation failed");
    int64_t n = 0;
    rc = HS_OK;
    if (hipMemcpyAsync(d + o_q, qc.data(), (size_t)qlen, hipMemcpyHostToDevice, st) != hipSuccess)
        rc = fail(HS_EDEVICE, "query copy failed");
    if (!rc)
        rc = launch_threshold(db, (const uint8_t*)(d + o_q), qlen, params, dcap, na, st, d + o_ws,
                              (DevHit*)(d + o_hits), (int64_t*)(d + o_n), (DevAln*)(d + o_alns),
                              (uint32_t*)(d + o_ops), stride);
    if (!rc && (hipMemcpyAsync(&n, d + o_n, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess))
        rc = fail(HS_EDEVICE, "threshold search failed on the device");
    const int64_t n_out = std::min<int64_t>(n, dcap);
    const int32_t n_a = (int32_t)std::min<int64_t>(na, n_out);
    std::vector<DevAln> h_alns((size_t)std::max(n_a, 1));
    std::vector<uint32_t> h_ops((size_t)stride * std::max(n_a, 1));
    if (!rc && n <= cap) {
        if ((n_out > 0 && hipMemcpyAsync(hits, d + o_hits, sizeof(DevHit) * (size_t)n_out,
                                         hipMemcpyDeviceToHost, st) != hipSuccess) ||
            (n_a > 0 && hipMemcpyAsync(h_alns.data(), d + o_alns, sizeof(DevAln) * n_a,
                                       hipMemcpyDeviceToHost, st) != hipSuccess) ||
            (n_a > 0 && hipMemcpyAsync(h_ops.data(), d + o_ops, sizeof(uint32_t) * stride * n_a,
                                       hipMemcpyDeviceToHost, st) != hipSuccess) ||
            hipStreamSynchronize(st) != hipSuccess)
            rc = fail(HS_EDEVICE, "threshold results copy failed");
    }
    (void)hipFreeAsync(d, st);
    if (rc) return rc;
    *n_hits = n;
    if (n > cap) return fail(HS_ENOSPC, "more targets reach the threshold than cap");
    if (n_aln > 0) {
        int64_t need = 0;
        for (int32_t i = 0; i < n_a; ++i) need += h_alns[(size_t)i].n_ops;
        *ops_used = need;
        if (need > ops_cap) return fail(HS_ENOSPC, "ops buffer too small");
        int64_t off = 0;
        for (int32_t i = 0; i < n_a; ++i) {
            const DevAln& a = h_alns[(size_t)i];
            std::memcpy(ops + off, h_ops.data() + a.ops_off, sizeof(uint32_t) * a.n_ops);
            alns[i].target_id = a.target_id;
            alns[i].score = a.score;
            alns[i].n_ops = a.n_ops;
            alns[i].ops_off = off;
            off += a.n_ops;
        }
        *n_alns = n_a;
    }
    return HS_OK;
}

namespace {

// Pairwise workspace: pair table, work order, per-round scores, pair counters.
struct AlignWs {
    size_t o_pairs, o_order, o_rs, o_done, total;
    AlignWs(int32_t n, int32_t rounds) {
        o_pairs = 0;
        o_order = align_up(sizeof(AlignPair) * (size_t)n);
        o_rs = o_order + align_up(sizeof(int32_t) * (size_t)n);
        o_done = o_rs + align_up(sizeof(int32_t) * (size_t)n * (size_t)rounds);
        total = o_done + align_up(sizeof(uint32_t) * (size_t)n);
    }
};

// Checks the pairs' lengths (host offsets) and fills their table: codes at
// qoff[i] / toff[i] relative to `base`, each pair's op slot after the
// previous pairs' (qlen + tlen entries each).  Returns the longest sequence
// in *longest.
int align_pairs_table(int32_t n, const int64_t* qoff, const int64_t* toff, const hs_params* params,
                      std::vector<AlignPair>& pairs, int64_t* longest) {
    if (n < 1 || n > HS_MAX_ALIGN_PAIRS) return fail(HS_EINVAL, "n must lie in [1, HS_MAX_ALIGN_PAIRS]");
    if (!qoff || !toff) return fail(HS_EINVAL, "NULL offsets");
    int rc = check_params(params);
    if (rc) return rc;
    if ((int64_t)n * params->rounds > 0x7FFFFFFF) return fail(HS_EINVAL, "n * rounds too large");
    pairs.resize((size_t)n);
    int64_t co = 0, lo = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int64_t a = qoff[i + 1] - qoff[i], b = toff[i + 1] - toff[i];
        if (a < 1 || a > HS_MAX_ALIGN || b < 1 || b > HS_MAX_ALIGN)
            return fail(HS_EINVAL, "pair " + std::to_string(i) + ": lengths must lie in [1, HS_MAX_ALIGN]");
        AlignPair& P = pairs[(size_t)i];
        P.qlen = (int32_t)a;
        P.tlen = (int32_t)b;
        P.qoff = qoff[i];
        P.toff = toff[i];
        P.ops_off = co;
        co += a + b;          // runs never outnumber columns
        lo = std::max(lo, std::max(a, b));
    }
    *longest = lo;
    return HS_OK;
}

// Queues the pairwise rounds and replays of the pairs (table `pairs`, codes
// relative to d_codes) on st, with the workspace at ws (AlignWs layout):
// scores, rounds (may be NULL), op counts and ops in the pairs' slots.
int align_queue(const std::vector<AlignPair>& pairs, int64_t longest, const uint8_t* d_codes,
                const hs_params* params, hipStream_t st, char* ws, int32_t* d_scores,
                int32_t* d_rounds, int32_t* d_n_ops, uint32_t* d_ops) {
    const int32_t n = (int32_t)pairs.size();
    const AlignWs L(n, params->rounds);
    // workgroups take the pairs with the most cells per round first (a
    // round's cells grow with the product of the lengths), so that the
    // longest chains of steps start at once
    std::vector<int32_t> order((size_t)n);
    for (int32_t i = 0; i < n; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return (int64_t)pairs[(size_t)a].qlen * pairs[(size_t)a].tlen >
               (int64_t)pairs[(size_t)b].qlen * pairs[(size_t)b].tlen;
    });
    if (hipMemcpyAsync(ws + L.o_pairs, pairs.data(), sizeof(AlignPair) * (size_t)n, hipMemcpyHostToDevice,
                       st) != hipSuccess ||
        hipMemcpyAsync(ws + L.o_order, order.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice,
                       st) != hipSuccess)
        return fail(HS_EDEVICE, "pair upload failed");
    hipLaunchKernelGGL(k_align_reset, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (uint32_t*)(ws + L.o_done), n);
    const KParams kp = kparams(params);
    const KMatrix km = kmatrix(params);
    const AlignPair* d_pairs = (const AlignPair*)(ws + L.o_pairs);
    const int32_t* d_order = (const int32_t*)(ws + L.o_order);
    int32_t* d_rs = (int32_t*)(ws + L.o_rs);
    uint32_t* d_done = (uint32_t*)(ws + L.o_done);
    const unsigned nr = (unsigned)((int64_t)n * params->rounds);
    // LDS sized to the longest sequence, so that batches of short pairs
    // keep many workgroups on a compute unit
    const int32_t cap = (int32_t)longest;
    const size_t lds = al_lds_bytes(cap);
    // a batch holding a pair of kAlLongPair letters or more gives each
    // (pair, round) 1,024 threads: a step of a long pair has thousands of
    // placements (the 5,600 x 5,600 pair at Rounds 20: 5.8 ms with 256
    // threads, 1.6 ms with 1,024, before the four placements per thread);
    // batches of shorter pairs take 128 threads, enough for the few
    // hundred placements of their steps (1,000 pairs of up to 2,000
    // letters: kernel 0.87 ms, against 1.07 with 256 threads taking one
    // placement each, 1.46 with 256 taking four, 1.23 with 64)
    if (longest >= kAlLongPair)
        hipLaunchKernelGGL(k_align_pairs<kAlThreadsLong>, dim3(nr), dim3(kAlThreadsLong), lds, st, d_pairs,
                           d_order, d_codes, cap, kp, km, d_rs, d_done, d_scores, d_rounds, d_n_ops, d_ops);
    else
        hipLaunchKernelGGL(k_align_pairs<kAlThreadsShort>, dim3(nr), dim3(kAlThreadsShort), lds, st, d_pairs,
                           d_order, d_codes, cap, kp, km, d_rs, d_done, d_scores, d_rounds, d_n_ops, d_ops);
    if (hipGetLastError() != hipSuccess) return fail(HS_EDEVICE, "pairwise kernel failed to launch");
    return HS_OK;
}

}  // namespace

int64_t hs_align_workspace_bytes(int32_t n, int32_t rounds) {
    if (n < 1 || n > HS_MAX_ALIGN_PAIRS || rounds < 1 || rounds > 1024) return 0;
    return (int64_t)AlignWs(n, rounds).total;
}

int hs_align_batch_dev(int32_t n, const uint8_t* d_codes, const int64_t* qoff, const int64_t* toff,
                       const hs_params* params, void* stream, void* d_ws, size_t ws_bytes,
                       int32_t* d_scores, int32_t* d_rounds, uint32_t* d_ops, int32_t* d_n_ops) {
    std::vector<AlignPair> pairs;
    int64_t longest = 0;
    int rc = align_pairs_table(n, qoff, toff, params, pairs, &longest);
    if (rc) return rc;
    if (!d_codes || !d_ws || !d_scores || !d_ops || !d_n_ops) return fail(HS_EINVAL, "NULL device pointer");
    if (ws_bytes < AlignWs(n, params->rounds).total) return fail(HS_ENOSPC, "workspace too small");
    return align_queue(pairs, longest, d_codes, params, (hipStream_t)stream, (char*)d_ws, d_scores,
                       d_rounds, d_n_ops, d_ops);
}

int hs_align_batch(int32_t n, const char* qres, const int64_t* qoff, const char* tres,
                   const int64_t* toff, const hs_params* params, void* stream, int32_t* scores,
                   int32_t* rounds, uint32_t* ops, int64_t ops_cap, int64_t* ops_off,
                   int64_t* ops_used) {
    if (!qres || !tres || !scores || !ops_off || !ops_used) return fail(HS_EINVAL, "NULL pointer");
    // the pairs' letters go to the device back to back, queries first: their
    // offsets there are the host offsets less the first, targets after the
    // queries
    std::vector<AlignPair> pairs;
    int64_t longest = 0;
    int rc = align_pairs_table(n, qoff, toff, params, pairs, &longest);
    if (rc) return rc;
    const int64_t nq = qoff[n] - qoff[0], nt = toff[n] - toff[0];
    for (AlignPair& P : pairs) {
        P.qoff -= qoff[0];
        P.toff += nq - toff[0];
    }
    const int64_t nops = nq + nt;
    std::vector<uint8_t> codes((size_t)(nq + nt));
    if ((rc = hs_encode(qres + qoff[0], nq, codes.data()))) return rc;
    if ((rc = hs_encode(tres + toff[0], nt, codes.data() + nq))) return rc;
    hipStream_t st = (hipStream_t)stream;
    // device layout: codes, the pairwise workspace, then one region of
    // scores, rounds and packed offsets (read back by one copy), op counts,
    // ops in per-pair slots, packed ops
    const AlignWs W(n, params->rounds);
    const size_t o_codes = 0, o_ws = align_up(codes.size()),
                 o_sc = o_ws + W.total,
                 o_rd = o_sc + sizeof(int32_t) * (size_t)n,
                 o_off = (o_rd + sizeof(int32_t) * (size_t)n + 7) & ~(size_t)7,
                 o_no = align_up(o_off + sizeof(int64_t) * ((size_t)n + 1)),
                 o_ops = o_no + align_up(sizeof(int32_t) * (size_t)n),
                 o_pk = o_ops + align_up(sizeof(uint32_t) * (size_t)nops),
                 total = o_pk + align_up(sizeof(uint32_t) * (size_t)nops);
    char* d = nullptr;
    if (hipMallocAsync((void**)&d, total, st) != hipSuccess)
        return fail(HS_ENOMEM, "device allocation failed");
    std::vector<char> h_head(o_no - o_sc);
    if (hipMemcpyAsync(d + o_codes, codes.data(), codes.size(), hipMemcpyHostToDevice, st) != hipSuccess)
        rc = fail(HS_EDEVICE, "letter upload failed");
    if (!rc)
        rc = align_queue(pairs, longest, (const uint8_t*)(d + o_codes), params, st, d + o_ws,
                         (int32_t*)(d + o_sc), (int32_t*)(d + o_rd), (int32_t*)(d + o_no),
                         (uint32_t*)(d + o_ops));
    if (!rc) {
        // pack: a scan over the pairs' op counts, then one wavefront per pair
        const AlignPair* d_pairs = (const AlignPair*)(d + o_ws + W.o_pairs);
        hipLaunchKernelGGL(k_align_ops_scan, dim3(1), dim3(kAlScanThreads), 0, st,
                           (const int32_t*)(d + o_no), n, (int64_t*)(d + o_off));
        hipLaunchKernelGGL(k_align_ops_pack, dim3((unsigned)((n + kAlWaves - 1) / kAlWaves)), dim3(kAlThreads),
                           0, st, d_pairs, n, (const int32_t*)(d + o_no), (const int64_t*)(d + o_off),
                           (const uint32_t*)(d + o_ops), (uint32_t*)(d + o_pk));
        if (hipGetLastError() != hipSuccess) rc = fail(HS_EDEVICE, "pairwise kernels failed to launch");
    }
    // scores, rounds and offsets first; then exactly the packed ops, straight
    // into the caller's buffer when they fit
    if (!rc && (hipMemcpyAsync(h_head.data(), d + o_sc, h_head.size(), hipMemcpyDeviceToHost, st) ||
                hipStreamSynchronize(st)))
        rc = fail(HS_EDEVICE, "pairwise alignment failed on the device");
    const int64_t* h_off = (const int64_t*)(h_head.data() + (o_off - o_sc));
    const int64_t need = rc ? 0 : h_off[n];
    if (!rc) {
        *ops_used = need;
        if (need > ops_cap) rc = fail(HS_ENOSPC, "ops buffer too small");
    }
    if (!rc && need > 0 && (!ops || hipMemcpyAsync(ops, d + o_pk, sizeof(uint32_t) * (size_t)need,
                                                   hipMemcpyDeviceToHost, st) ||
                            hipStreamSynchronize(st)))
        rc = fail(HS_EDEVICE, "pairwise alignment ops copy failed");
    (void)hipFreeAsync(d, st);
    if (rc) return rc;
    std::memcpy(ops_off, h_off, sizeof(int64_t) * ((size_t)n + 1));
    std::memcpy(scores, h_head.data(), sizeof(int32_t) * (size_t)n);
    if (rounds) std::memcpy(rounds, h_head.data() + (o_rd - o_sc), sizeof(int32_t) * (size_t)n);
    return HS_OK;
}

int hs_align(const char* query, int32_t qlen, const char* target, int32_t tlen,
             const hs_params* params, void* stream, int32_t* score, int32_t* round, uint32_t* ops,
             int64_t ops_cap, int64_t* n_ops) {
    if (!score || !n_ops) return fail(HS_EINVAL, "NULL pointer");
    const int64_t qo[2] = {0, qlen}, to[2] = {0, tlen};
    int64_t off[2] = {0, 0};
    if (qlen < 1 || tlen < 1) return fail(HS_EINVAL, "lengths must lie in [1, HS_MAX_ALIGN]");
    return hs_align_batch(1, query, qo, target, to, params, stream, score, round, ops, ops_cap, off,
                          n_ops);
}

int64_t hs_sw_workspace_bytes(const hs_db* db) {
    if (!db) return fail(HS_EINVAL, "db is NULL");
    return (int64_t)align_up(sizeof(int2) * (size_t)std::max<int64_t>(db->n_residues, 1));
}

int hs_sw_scores_dev(const hs_db* db, const uint8_t* d_qcodes, int32_t qlen, const hs_params* params,
                     void* stream, void* d_ws, size_t ws_bytes, int32_t* d_scores) {
    if (!db) return fail(HS_EINVAL, "db is NULL");
    if (qlen < 1 || qlen > HS_MAX_QUERY) return fail(HS_EINVAL, "qlen must lie in [1, HS_MAX_QUERY]");
    int rc = check_params(params);
    if (rc) return rc;
    if (!d_qcodes || !d_scores || !d_ws) return fail(HS_EINVAL, "NULL device pointer");
    if ((int64_t)ws_bytes < hs_sw_workspace_bytes(db)) return fail(HS_ENOSPC, "workspace too small");
    if (db->n_targets < 1) return HS_OK;
    const int32_t qp = sw_profile_stride(qlen);
    const size_t lds = (size_t)kNsym * (size_t)qp;
    const void* fn = (const void*)k_sw_scores;
    if ((rc = set_lds_limit(fn, lds))) return rc;
    const int64_t lane_passes = (qlen + kSwRows - 1) / kSwRows;
    const int64_t wave_passes = (qlen + kSwWaveRows - 1) / kSwWaveRows;
    const int32_t G = sw_group_lanes(qlen);
    // Queries of one pass: a group of G lanes sweeps a target in tlen + G - 1
    // steps against the lane role's G passes of tlen steps with a boundary
    // written and read between passes, so every target of at least
    // kSwGroupMin * G letters takes a group (the full workload: 61.5 ms when
    // one target held a wavefront whatever the query's length, 20.3 ms from
    // 2 G letters on, 19.9 ms from G on).  Longer queries: targets whose
    // one-lane sweep would outlast half the wavefront sweep of the longest
    // target take a wavefront each (at half the threshold the lanes near it,
    // which share their SIMDs, ran 62 ms instead of 72; a quarter gained nothing).
    const int64_t thr = G < kLanes ? (int64_t)kSwGroupMin * G - 1
                                   : wave_passes * ((int64_t)db->lens_desc[0] + kLanes - 1) /
                                         (2 * lane_passes);
    const int32_t n_long = (int32_t)(std::partition_point(db->lens_desc.begin(), db->lens_desc.end(),
                                                          [&](int32_t L) { return L > thr; }) -
                                     db->lens_desc.begin());
    const int64_t per_block = (int64_t)(kSwThreads / kLanes) * (kLanes / G);
    const int64_t wave_blocks = (n_long + per_block - 1) / per_block;
    const int64_t grid = wave_blocks + (db->n_targets - n_long + kSwThreads - 1) / kSwThreads;
    hipLaunchKernelGGL(k_sw_scores, dim3((unsigned)grid), dim3(kSwThreads), lds, (hipStream_t)stream,
                       db->view(), n_long, d_qcodes, qlen, qp, kmatrix(params), params->gop,
                       params->gep, (int2*)d_ws, d_scores);
    HIP_TRY(hipGetLastError());
    return HS_OK;
}

int hs_batch_create(const hs_db* db, int32_t max_nq, int32_t max_qlen, int64_t max_residues,
                    int32_t k, int32_t n_aln, hs_batch** out) {
    if (!out) return fail(HS_EINVAL, "out is NULL");
    if (!db) return fail(HS_EINVAL, "db is NULL");
    if (max_nq < 1 || max_nq > HS_MAX_BATCH) return fail(HS_EINVAL, "max_nq must lie in [1, HS_MAX_BATCH]");
    if (max_qlen < 1 || max_qlen > HS_MAX_QUERY)
        return fail(HS_EINVAL, "max_qlen must lie in [1, HS_MAX_QUERY]");
    if (max_residues < 1 || max_residues > (int64_t)max_nq * max_qlen)
        return fail(HS_EINVAL, "max_residues must lie in [1, max_nq * max_qlen]");
    if (k < 1 || k > HS_MAX_K) return fail(HS_EINVAL, "k must lie in [1, HS_MAX_K]");
    if (n_aln < 0 || n_aln > k) return fail(HS_EINVAL, "n_aln must lie in [0, k]");
    if (!copies_fit(max_qlen, 1)) return fail(HS_EINVAL, "max_qlen too long for the device's LDS");
    hs_batch* b = new hs_batch();
    b->db = db;
    b->max_nq = max_nq;
    b->max_qlen = max_qlen;
    b->max_res = max_residues;
    b->k = k;
    b->n_aln = n_aln;
    b->ops_stride = 2 * (int64_t)max_qlen + 2;
    const int64_t chunks = (db->n_queue + min_chunk(db) - 1) / min_chunk(db);
    // items of min_chunk positions, or for a small batch one position per
    // wavefront, up to two workgroups per compute unit
    b->max_items = std::max<int64_t>((int64_t)max_nq * std::max<int64_t>(chunks, 1),
                                     2 * (int64_t)device_cus());
    // one item per query, or for a small batch up to two per compute unit
    b->max_titems = std::max<int64_t>((int64_t)max_nq, 2 * (int64_t)device_cus());
    const size_t nt = (size_t)std::max<int64_t>(db->n_targets, 1);
    const size_t nal = (size_t)max_nq * (size_t)std::max(n_aln, 1);
    // one device allocation, carved below
    size_t sz[20];
    int ns = 0;
    sz[ns++] = align_up((size_t)max_residues);                                // codes
    sz[ns++] = align_up(sizeof(BatchQuery) * max_nq);
    sz[ns++] = align_up(sizeof(KMatrix) * max_nq);
    sz[ns++] = align_up(sizeof(BatchItem) * (size_t)b->max_items);
    sz[ns++] = align_up(sizeof(BatchItem) * (size_t)b->max_titems);
    sz[ns++] = kAlign;                                                        // counters
    sz[ns++] = align_up(sizeof(int32_t) * nt * max_nq);                       // scores
    sz[ns++] = align_up(sizeof(int32_t) * nt * max_nq);                       // rounds
    sz[ns++] = align_up(sizeof(uint64_t) * 8 * (size_t)std::max<int64_t>(db->n_queue, 1));
    sz[ns++] = align_up(sizeof(TopkState) * max_nq);
    sz[ns++] = align_up(sizeof(uint32_t) * kWinBins * max_nq);
    sz[ns++] = align_up(sizeof(uint64_t) * kSortCap * max_nq);
    sz[ns++] = align_up(sizeof(DevHit) * (size_t)k * max_nq);
    sz[ns++] = align_up(sizeof(int32_t) * max_nq);
    sz[ns++] = align_up(sizeof(DevAln) * nal);
    sz[ns++] = align_up(sizeof(uint32_t) * nal * (size_t)b->ops_stride);      // ops
    sz[ns++] = align_up(sizeof(int64_t) * (nal + 1)) + align_up(sizeof(uint32_t) * nal * (size_t)b->ops_stride);
    size_t total = 0;
    for (int i = 0; i < ns; ++i) total += sz[i];
    if (hipMalloc((void**)&b->d_mem, total) != hipSuccess) {
        b->d_mem = nullptr;
        free_batch(b);
        return fail(HS_ENOMEM, "device allocation of " + std::to_string(total) + " bytes for the batch failed");
    }
    char* p = b->d_mem;
    int i = 0;
    b->d_qcodes = (uint8_t*)p; p += sz[i++];
    b->d_qs = (BatchQuery*)p; p += sz[i++];
    b->d_mats = (KMatrix*)p; p += sz[i++];
    b->d_items = (BatchItem*)p; p += sz[i++];
    b->d_titems = (BatchItem*)p; p += sz[i++];
    b->d_ctr = (uint32_t*)p; p += sz[i++];
    b->d_scores = (int32_t*)p; p += sz[i++];
    b->d_rounds = (int32_t*)p; p += sz[i++];
    b->d_draws = (uint64_t*)p; p += sz[i++];
    b->d_st = (TopkState*)p; p += sz[i++];
    b->d_hist = (uint32_t*)p; p += sz[i++];
    b->d_keys = (uint64_t*)p; p += sz[i++];
    b->d_hits = (DevHit*)p; p += sz[i++];
    b->d_n_hits = (int32_t*)p; p += sz[i++];
    b->d_alns = (DevAln*)p; p += sz[i++];
    b->d_ops = (uint32_t*)p; p += sz[i++];
    b->d_pos = (int64_t*)p;
    b->d_packed = (uint32_t*)(p + align_up(sizeof(int64_t) * (nal + 1)));
    const size_t up = sz[0] + sz[1] + sz[2] + sz[3] + sz[4];
    // the packing offsets and, right after them as on the device, up to
    // 64 KB of packed ops: results that small come back in one copy
    b->ops_prefix = std::min<size_t>(sizeof(uint32_t) * nal * (size_t)b->ops_stride, 64 * 1024);
    // (plus slack: the copy kernel moves whole 16-byte words)
    const size_t down = sz[12] + sz[13] + sz[14] + align_up(sizeof(int64_t) * (nal + 1)) +
                        align_up(b->ops_prefix);
    void* up_view = nullptr;
    void* down_view = nullptr;
    if (hipHostMalloc((void**)&b->h_up, up, hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc((void**)&b->h_down, down, hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer(&up_view, b->h_up, 0) != hipSuccess ||
        hipHostGetDevicePointer(&down_view, b->h_down, 0) != hipSuccess) {
        free_batch(b);
        return fail(HS_ENOMEM, "pinned host allocation for the batch failed");
    }
    b->d_up_view = (const char*)up_view;
    b->d_down_view = (char*)down_view;
    b->h_qcodes = (uint8_t*)b->h_up;
    b->h_qs = (BatchQuery*)(b->h_up + sz[0]);
    b->h_mats = (KMatrix*)(b->h_up + sz[0] + sz[1]);
    b->h_items = (BatchItem*)(b->h_up + sz[0] + sz[1] + sz[2]);
    b->h_titems = (BatchItem*)(b->h_up + sz[0] + sz[1] + sz[2] + sz[3]);
    b->h_hits = (DevHit*)b->h_down;
    b->h_nh = (int32_t*)(b->h_down + sz[12]);
    b->h_alns = (DevAln*)(b->h_down + sz[12] + sz[13]);
    b->h_pos = (int64_t*)(b->h_down + sz[12] + sz[13] + sz[14]);
    b->h_packed = (uint32_t*)((char*)b->h_pos + align_up(sizeof(int64_t) * (nal + 1)));
    // resolve every kernel a search of the batch may launch now, rather than
    // on the first search that needs it
    const void* fns[] = {
        (const void*)k_score_batch<4, false, false>, (const void*)k_score_batch<4, false, true>,
        (const void*)k_score_batch<1, false, false>, (const void*)k_score_batch<1, false, true>,
        (const void*)k_score_one<4, false>, (const void*)k_score_one<1, false>,
        (const void*)k_trace_batch<4>, (const void*)k_trace_batch<1>};
    for (const void* fn : fns) {
        hipFuncAttributes attr;
        (void)hipFuncGetAttributes(&attr, fn);
    }
    *out = b;
    return HS_OK;
}

int hs_batch_free(hs_batch* b) {
    free_batch(b);
    return HS_OK;
}

int hs_batch_set(hs_batch* b, int32_t nq, const char* residues, const int64_t* offsets,
                 const hs_params* params, int32_t n_params, void* stream) {
    if (!b) return fail(HS_EINVAL, "batch is NULL");
    if (nq < 1 || nq > b->max_nq) return fail(HS_EINVAL, "nq must lie in [1, max_nq]");
    if (!residues || !offsets || !params) return fail(HS_EINVAL, "NULL residues, offsets or params");
    if (n_params != 1 && n_params != nq) return fail(HS_EINVAL, "n_params must be 1 or nq");
    hipStream_t st = (hipStream_t)stream;
    const int64_t total = offsets[nq] - offsets[0];
    if (total < 1 || total > b->max_res) return fail(HS_EINVAL, "total query length must lie in [1, max_residues]");
    std::vector<int32_t> qlens((size_t)nq);
    int32_t mx = 0;
    for (int32_t q = 0; q < nq; ++q) {
        const int64_t L = offsets[q + 1] - offsets[q];
        if (L < 1 || L > b->max_qlen)
            return fail(HS_EINVAL, "query " + std::to_string(q) + " has length outside [1, max_qlen]");
        qlens[(size_t)q] = (int32_t)L;
        mx = std::max(mx, (int32_t)L);
    }
    for (int32_t i = 0; i < n_params; ++i) {
        int rc = check_params(params + i);
        if (rc) return rc;
    }
    // the pinned mirror is free: every earlier upload completed before its
    // hs_batch_set (or hs_batch_schedule) returned
    uint8_t* codes = b->h_qcodes;
    {
        int rc = hs_encode(residues + offsets[0], total, codes);
        if (rc) return rc;
    }
    const uint64_t seed0 = params[0].seed;
    const bool new_table = !b->table_valid || b->table_seed != seed0;
    BatchQuery* qs = b->h_qs;
    KMatrix* mats = b->h_mats;
    for (int32_t q = 0; q < nq; ++q) {
        const hs_params* p = params + (n_params == 1 ? 0 : q);
        BatchQuery& Q = qs[(size_t)q];
        Q.kp = kparams(p);
        Q.qoff = offsets[q] - offsets[0];
        Q.qlen = qlens[(size_t)q];
        mats[(size_t)q] = kmatrix(p);
        Q.bias = matrix_bias(mats[(size_t)q]);
        Q.table = p->seed == seed0 ? 1 : 0;
        Q.pad_ = 0;
    }
    b->nq = 0;      // not usable until the upload below completes
    drop_graph(b);
    // codes, queries and matrices (their device regions lie at the mirror's
    // offsets); the work items follow in upload_items, which waits for both
    {
        const int64_t off[3] = {0, (const char*)qs - b->h_up, (const char*)mats - b->h_up};
        const int64_t len[3] = {total, (int64_t)sizeof(BatchQuery) * nq, (int64_t)sizeof(KMatrix) * nq};
        if (int rc = pull_segments(b, st, off, len, 3)) return rc;
    }
    if (new_table && b->db->n_queue > 0) {
        const int32_t nqueue = (int32_t)b->db->n_queue;
        hipLaunchKernelGGL(k_draws, dim3((2 * (int64_t)nqueue + 255) / 256), dim3(256), 0, st,
                           (const PairRec*)b->db->d_recs, nqueue, seed0, b->d_draws, b->d_ctr,
                           TopkWs{}, 0, 0);
        HIP_TRY(hipGetLastError());
    }
    b->table_valid = true;
    b->table_seed = seed0;
    b->nq = nq;
    b->qlens = qlens;
    b->cur_max_qlen = mx;
    int rc = choose_schedule(b, st);
    if (rc) {
        b->nq = 0;
        (void)hipStreamSynchronize(st);     // the mirror may be rewritten after return
    }
    return rc;
}

int hs_batch_schedule(hs_batch* b, int32_t copies, int32_t cap, int32_t chunk, void* stream) {
    if (!b) return fail(HS_EINVAL, "batch is NULL");
    if (copies != 0 && copies != 1 && copies != 4) return fail(HS_EINVAL, "copies must be 0, 1 or 4");
    if (cap < 0 || cap > kLanes) return fail(HS_EINVAL, "cap must lie in [0, 64]");
    if (chunk < 0 || chunk % 64 != 0) return fail(HS_EINVAL, "chunk must be 0 or a positive multiple of 64");
    if (copies == 4 && b->nq > 0 && !copies_fit(b->cur_max_qlen, 4))
        return fail(HS_EINVAL, "four profile copies do not fit in LDS for the longest query");
    b->fix_copies = copies;
    b->fix_cap = cap;
    b->fix_chunk = chunk;
    if (b->nq < 1) return HS_OK;
    return choose_schedule(b, (hipStream_t)stream);
}

int hs_batch_get_schedule(const hs_batch* b, int32_t* copies, int32_t* cap, int32_t* chunk,
                          int32_t* grid, int32_t* n_items) {
    if (!b) return fail(HS_EINVAL, "batch is NULL");
    if (copies) *copies = b->copies;
    if (cap) *cap = b->cap;
    if (chunk) *chunk = b->chunk;
    if (grid) *grid = b->grid;
    if (n_items) *n_items = b->n_items;
    return HS_OK;
}

int hs_batch_get_launch(const hs_batch* b, int32_t* record, int32_t* waves, int32_t* ilp,
                        int32_t* one_pair) {
    int rc = check_batch_ready(b);
    if (rc) return rc;
    if (record) *record = b->score_one ? 0 : b->rec;
    if (waves) *waves = b->score_one ? b->waves : b->swaves;
    if (ilp) *ilp = b->score_one ? 0 : (int32_t)b->ilp;
    if (one_pair) *one_pair = b->score_one ? 1 : 0;
    return HS_OK;
}

int hs_batch_tune(hs_batch* b, void* stream, int32_t reps, float* best_ms) {
    int rc = check_batch_ready(b);
    if (rc) return rc;
    if (reps < 1) reps = 1;
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> copies_c = {1};
    if (copies_fit(b->cur_max_qlen, 4)) copies_c.push_back(4);
    const int32_t full = (int32_t)round64(std::max<int64_t>(b->db->n_queue, 64));
    std::vector<int32_t> chunk_c;
    for (int32_t c = full; c >= min_chunk(b->db); c /= 2) {
        const int32_t r = (int32_t)round64(c);
        if (chunk_c.empty() || chunk_c.back() != r) chunk_c.push_back(r);
        if (c <= 64) break;
    }
    const int32_t cap_c[] = {4, 8, 16, 32, 64};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(HS_EDEVICE, "event creation failed");
    }
    float best = 1e30f;
    int32_t bc = 0, bk = 0, bch = 0;
    // mean time of `reps` scoring passes under one schedule, after a warm-up
    auto time_one = [&](int32_t cp, int32_t ca, int32_t ch, float* ms) -> int {
        b->fix_copies = cp;
        b->fix_cap = ca;
        b->fix_chunk = ch;
        int r = choose_schedule(b, st);
        if (!r) r = enqueue_batch_score(b, st, nullptr);
        if (r) return r;
        if (hipEventRecord(e0, st) != hipSuccess) return fail(HS_EDEVICE, "event record failed");
        for (int32_t i = 0; i < reps && !r; ++i) r = enqueue_batch_score(b, st, nullptr);
        if (r) return r;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(ms, e0, e1) != hipSuccess)
            return fail(HS_EDEVICE, "timing failed");
        *ms /= (float)reps;
        return HS_OK;
    };
    for (int32_t cp : copies_c) {
        for (int32_t ca : cap_c) {
            for (int32_t ch : chunk_c) {
                float ms = 0;
                if ((rc = time_one(cp, ca, ch, &ms))) break;
                if (ms < best) {
                    best = ms;
                    bc = cp;
                    bk = ca;
                    bch = ch;
                }
            }
            if (rc) break;
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        b->fix_copies = b->fix_cap = b->fix_chunk = 0;
        (void)choose_schedule(b, st);
        return rc;
    }
    b->fix_copies = bc;
    b->fix_cap = bk;
    b->fix_chunk = bch;
    if ((rc = choose_schedule(b, st))) return rc;
    if (best_ms) *best_ms = best;
    return HS_OK;
}

int hs_batch_score(hs_batch* b, void* stream, uint64_t* d_cells) {
    int rc = check_batch_ready(b);
    if (rc) return rc;
    return enqueue_batch_score(b, (hipStream_t)stream, d_cells);
}

int hs_batch_run(hs_batch* b, void* stream) {
    int rc = check_batch_ready(b);
    if (rc) return rc;
    return enqueue_batch(b, (hipStream_t)stream);
}

int hs_batch_run_graph(hs_batch* b, void* stream) {
    int rc = check_batch_ready(b);
    if (rc) return rc;
    if (!b->exec) {
        if (!b->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        rc = enqueue_batch(b, b->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
        if (rc || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return rc ? rc : fail(HS_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(e));
        }
        const hipError_t ei = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            b->exec = nullptr;
            return fail(HS_EDEVICE, std::string("graph instantiation failed: ") + hipGetErrorString(ei));
        }
    }
    HIP_TRY(hipGraphLaunch(b->exec, (hipStream_t)stream));
    return HS_OK;
}

int hs_batch_outputs(const hs_batch* b, hs_hit** d_hits, int32_t** d_n_hits, hs_aln** d_alns,
                     uint32_t** d_ops, int64_t* ops_stride, int32_t** d_scores, int32_t** d_rounds) {
    if (!b) return fail(HS_EINVAL, "batch is NULL");
    if (d_hits) *d_hits = (hs_hit*)b->d_hits;
    if (d_n_hits) *d_n_hits = b->d_n_hits;
    if (d_alns) *d_alns = (hs_aln*)b->d_alns;
    if (d_ops) *d_ops = b->d_ops;
    if (ops_stride) *ops_stride = b->ops_stride;
    if (d_scores) *d_scores = b->d_scores;
    if (d_rounds) *d_rounds = b->d_rounds;
    return HS_OK;
}

int hs_batch_results(hs_batch* b, void* stream, hs_hit* hits, int32_t* n_hits, hs_aln* alns,
                     int32_t* n_alns, uint32_t* ops, int64_t ops_cap, int64_t* ops_used) {
    int rc = check_batch_ready(b);
    if (rc) return rc;
    if (!hits || !n_hits || (b->n_aln > 0 && (!alns || !n_alns || !ops_used)))
        return fail(HS_EINVAL, "NULL output pointer");
    hipStream_t st = (hipStream_t)stream;
    const int32_t nq = b->nq, k = b->k, na = b->n_aln;
    // pinned mirrors of the result regions (hits, counts and alignments lie
    // back to back on the device, as in the mirror)
    const DevHit* h_hits = b->h_hits;
    const int32_t* h_nh = b->h_nh;
    const DevAln* h_alns = b->h_alns;
    const int64_t* h_pos = b->h_pos;
    if (na > 0) {
        hipLaunchKernelGGL(k_ops_scan, dim3(1), dim3(1024), 0, st, (const DevAln*)b->d_alns,
                           (const int32_t*)b->d_n_hits, nq, na, b->d_pos);
        hipLaunchKernelGGL(k_ops_gather, dim3(na, nq), dim3(64), 0, st, (const DevAln*)b->d_alns,
                           (const int32_t*)b->d_n_hits, na, (const uint32_t*)b->d_ops,
                           (const int64_t*)b->d_pos, b->d_packed);
        HIP_TRY(hipGetLastError());
    }
    // hits, counts and alignments (back to back on the device and in the
    // mirror); packing offsets and the packed ops' first ops_prefix bytes
    const size_t span = na > 0 ? (size_t)((const char*)(h_alns + (size_t)nq * na) - (const char*)h_hits)
                               : (size_t)((const char*)(h_nh + nq) - (const char*)h_hits);
    {
        const int64_t soff[2] = {(const char*)b->d_hits - b->d_mem, (const char*)b->d_pos - b->d_mem};
        const int64_t doff[2] = {0, (const char*)b->h_pos - b->h_down};
        const int64_t len[2] = {(int64_t)span,
                                na > 0 ? (int64_t)((const char*)b->h_packed - (const char*)b->h_pos) +
                                             (int64_t)b->ops_prefix
                                       : 0};
        if ((rc = copy_segments(b->d_mem, b->d_down_view, st, soff, doff, len, 2))) return rc;
    }
    HIP_TRY(hipStreamSynchronize(st));
    if (na > 0) {
        const int64_t need = h_pos[(size_t)nq * na];
        *ops_used = need;
        if (need > ops_cap) return fail(HS_ENOSPC, "ops buffer too small");
        if (need > 0 && (size_t)need * sizeof(uint32_t) <= b->ops_prefix) {
            std::memcpy(ops, b->h_packed, sizeof(uint32_t) * (size_t)need);
        } else if (need > 0) {
            HIP_TRY(hipMemcpyAsync(ops, b->d_packed, sizeof(uint32_t) * need, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
    }
    for (int32_t q = 0; q < nq; ++q) {
        const int32_t nh = h_nh[(size_t)q];
        std::memcpy(hits + (size_t)q * k, h_hits + (size_t)q * k, sizeof(DevHit) * (size_t)nh);
        n_hits[q] = nh;
        if (na > 0) {
            const int32_t m = std::min(na, nh);
            for (int32_t a = 0; a < m; ++a) {
                const size_t i = (size_t)q * na + a;
                alns[i].target_id = h_alns[i].target_id;
                alns[i].score = h_alns[i].score;
                alns[i].n_ops = h_alns[i].n_ops;
                alns[i].ops_off = h_pos[i];
            }
            n_alns[q] = m;
        }
    }
    return HS_OK;
}

int hs_batch_scores(hs_batch* b, void* stream, int32_t* scores, int32_t* rounds) {
    int rc = check_batch_ready(b);
    if (rc) return rc;
    if (!scores) return fail(HS_EINVAL, "scores is NULL");
    hipStream_t st = (hipStream_t)stream;
    const size_t n = (size_t)b->nq * (size_t)b->db->n_targets;
    if (n) {
        HIP_TRY(hipMemcpyAsync(scores, b->d_scores, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
        if (rounds)
            HIP_TRY(hipMemcpyAsync(rounds, b->d_rounds, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    return HS_OK;
}

int hs_search_batch(const hs_db* db, int32_t nq, const char* residues, const int64_t* offsets,
                    const hs_params* params, int32_t n_params, int32_t k, int32_t n_aln,
                    void* stream, hs_hit* hits, int32_t* n_hits, hs_aln* alns, int32_t* n_alns,
                    uint32_t* ops, int64_t ops_cap, int64_t* ops_used) {
    if (!db) return fail(HS_EINVAL, "db is NULL");
    if (nq < 1 || nq > HS_MAX_BATCH) return fail(HS_EINVAL, "nq must lie in [1, HS_MAX_BATCH]");
    if (!offsets || !residues) return fail(HS_EINVAL, "NULL residues or offsets");
    int32_t mx = 1;
    for (int32_t q = 0; q < nq; ++q) {
        const int64_t L = offsets[q + 1] - offsets[q];
        if (L < 1 || L > HS_MAX_QUERY)
            return fail(HS_EINVAL, "query " + std::to_string(q) + " has length outside [1, HS_MAX_QUERY]");
        mx = std::max(mx, (int32_t)L);
    }
    hs_batch* b = nullptr;
    int rc = hs_batch_create(db, nq, mx, offsets[nq] - offsets[0], k, n_aln, &b);
    if (rc) return rc;
    rc = hs_batch_set(b, nq, residues, offsets, params, n_params, stream);
    if (!rc) rc = hs_batch_run(b, stream);
    if (!rc) rc = hs_batch_results(b, stream, hits, n_hits, alns, n_alns, ops, ops_cap, ops_used);
    free_batch(b);
    return rc;
}

const char* hs_last_error(void) { return g_err.c_str(); }

}  // extern "C"
