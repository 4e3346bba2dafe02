// hs_lib.hip -- host side of the C ABI declared in include/hs.h: database
// loading and packing, argument checking, kernel launches and result
// marshalling.  Everything the search computes runs in the kernels of the
// headers included below.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hs.h"
#include "device_common.hpp"
#include "score_kernels.hpp"
#include "topk_kernels.hpp"
#include "traceback_kernels.hpp"

using namespace hs;

static_assert(sizeof(hs_hit) == sizeof(DevHit), "hit layout");
static_assert(sizeof(hs_aln) == sizeof(DevAln), "alignment layout");

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

// --------------------------------------------------------------------------
// database image
// --------------------------------------------------------------------------
struct hs_db {
    int64_t n_targets = 0;
    int64_t n_residues = 0;
    uint8_t* d_letters = nullptr;   // codes, index order, kLetterPad readable bytes after
    int64_t* d_offsets = nullptr;
    int32_t* d_lens = nullptr;
    int32_t* d_order = nullptr;     // longest first
    PairRec* d_recs = nullptr;      // (index, length, offset) in hand-out order
    int64_t n_queue = 0;            // hand-out positions (targets plus padding)
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

namespace {

void free_db(hs_db* db) {
    if (!db) return;
    (void)hipFree(db->d_letters);
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

int set_lds_limit(const void* fn, size_t bytes) {
    if (bytes > 64 * 1024)
        HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
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

template <int kCopies, bool kCount>
int launch_sched(const hs_db* db, const uint8_t* d_q, int32_t qlen, const KParams& kp,
                 const KMatrix& km, int32_t bias, hipStream_t st, const QueryWs& w,
                 int32_t* d_scores, int32_t* d_rounds, uint64_t* d_cells, int32_t* d_max) {
    const void* fn = (const void*)k_score_sched<kCopies, kCount>;
    const size_t lds = sched_lds_bytes(qlen, kCopies);
    int rc = set_lds_limit(fn, lds);
    if (rc) return rc;
    int per_cu = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, lds));
    if (per_cu < 1) return fail(HS_ENOMEM, "scoring kernel does not fit on a compute unit");
    // every workgroup should get at least a quarter of its slots filled
    // every wavefront should get at least a quarter of its slots filled
    const int64_t want = (db->n_targets + kThreads / 4 - 1) / (kThreads / 4);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)per_cu * device_cus(), want));
    hipLaunchKernelGGL((k_score_sched<kCopies, kCount>), dim3(grid), dim3(kThreads), lds, st,
                       (const PairRec*)db->d_recs, (int32_t)db->n_queue, db->d_letters, d_q, qlen,
                       kp, km, bias, (const uint64_t*)w.draws, w.queue, d_scores, d_rounds,
                       (unsigned long long*)d_cells, d_max);
    HIP_TRY(hipGetLastError());
    return HS_OK;
}

int launch_score(const hs_db* db, const uint8_t* d_q, int32_t qlen, const hs_params* p,
                 hipStream_t st, const QueryWs& w, int32_t* d_scores, int32_t* d_rounds,
                 uint64_t* d_cells, int32_t* d_max) {
    if (db->n_targets == 0) return HS_OK;
    const KParams kp = kparams(p);
    const KMatrix km = kmatrix(p);
    const int32_t bias = matrix_bias(km);
    const int32_t nq = (int32_t)db->n_queue;
    hipLaunchKernelGGL(k_draws, dim3((nq + 255) / 256), dim3(256), 0, st, (const PairRec*)db->d_recs, nq,
                       kp.seed, w.draws, w.queue);
    HIP_TRY(hipGetLastError());
    const bool four = sched_lds_bytes(qlen, 4) <= device_lds_limit();
    if (!four && sched_lds_bytes(qlen, 1) > device_lds_limit())
        return fail(HS_EINVAL, "query too long for the device's LDS");
    if (d_cells)
        return four ? launch_sched<4, true>(db, d_q, qlen, kp, km, bias, st, w, d_scores, d_rounds, d_cells, d_max)
                    : launch_sched<1, true>(db, d_q, qlen, kp, km, bias, st, w, d_scores, d_rounds, d_cells, d_max);
    return four ? launch_sched<4, false>(db, d_q, qlen, kp, km, bias, st, w, d_scores, d_rounds, nullptr, d_max)
                : launch_sched<1, false>(db, d_q, qlen, kp, km, bias, st, w, d_scores, d_rounds, nullptr, d_max);
}

// Ranking of nq score arrays (query q's scores at scores + q * stride).
int launch_rank(const hs_db* db, hipStream_t st, const int32_t* scores, const int32_t* rounds,
                int64_t stride, int32_t nq, int32_t min_score, int32_t k, const TopkWs& tw,
                DevHit* d_hits, int32_t* d_n_hits) {
    const int32_t n = (int32_t)db->n_targets;
    const int tb = std::max(1, std::min(512, (n + 255) / 256));
    hipLaunchKernelGGL(k_topk_hist, dim3(tb, nq), dim3(256), 0, st, scores, stride, n, min_score, tw);
    hipLaunchKernelGGL(k_topk_pick, dim3(1, nq), dim3(256), 0, st, k, min_score, n, tw);
    hipLaunchKernelGGL(k_topk_collect, dim3(tb, nq), dim3(256), 0, st, scores, stride, n, min_score, tw);
    const size_t lds = sizeof(uint64_t) * kSortCap;
    int rc = set_lds_limit((const void*)k_topk_final, lds);
    if (rc) return rc;
    hipLaunchKernelGGL(k_topk_final, dim3(1, nq), dim3(1024), lds, st, scores, stride, rounds, n,
                       min_score, k, tw, d_hits, d_n_hits);
    HIP_TRY(hipGetLastError());
    return HS_OK;
}

// Queues one search.  All pointers are device pointers.
int launch_search(const hs_db* db, const uint8_t* d_q, int32_t qlen, const hs_params* p, int32_t k,
                  int32_t n_aln, hipStream_t st, void* d_ws, DevHit* d_hits, int32_t* d_n_hits,
                  DevAln* d_alns, uint32_t* d_ops, int64_t ops_stride) {
    QueryWs w = carve(d_ws, db->n_targets, db->n_queue);
    const int32_t n = (int32_t)db->n_targets;
    hipLaunchKernelGGL(k_topk_reset, dim3(1, 1), dim3(256), 0, st, w.tw());
    int rc = launch_score(db, d_q, qlen, p, st, w, w.scores, w.rounds, nullptr, &w.topk->max_score);
    if (rc) return rc;
    rc = launch_rank(db, st, w.scores, w.rounds, 0, 1, p->min_score, k, w.tw(), d_hits, d_n_hits);
    if (rc) return rc;
    if (n_aln > 0) {
        const KParams kp = kparams(p);
        const KMatrix km = kmatrix(p);
        const size_t lds = (size_t)profile_copy_bytes(profile_stride(qlen));
        rc = set_lds_limit((const void*)k_traceback, lds);
        if (rc) return rc;
        hipLaunchKernelGGL(k_traceback, dim3(n_aln), dim3(64), lds, st, db->view(), d_q, qlen, kp, km,
                           matrix_bias(km), d_hits, d_n_hits, n_aln, d_alns, d_ops, ops_stride);
        HIP_TRY(hipGetLastError());
    }
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

void hs_builtin_matrix(int8_t* out) {
    if (out) std::memcpy(out, kBlosum62, sizeof(kBlosum62));
}

int hs_encode(const char* ascii, int64_t n, uint8_t* codes) {
    if (n < 0 || (n > 0 && (!ascii || !codes))) return fail(HS_EINVAL, "bad arguments to hs_encode");
    for (int64_t i = 0; i < n; ++i) {
        const int c = kCodes.t[(unsigned char)ascii[i]];
        if (c < 0) return fail(HS_EINVAL, "residue outside the alphabet at position " + std::to_string(i));
        codes[i] = (uint8_t)c;
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

const char* hs_last_error(void) { return g_err.c_str(); }

}  // extern "C"
