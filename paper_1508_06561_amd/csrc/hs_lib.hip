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
    int32_t n_groups = 0;
    int64_t n_words = 0;
    uint32_t* d_words = nullptr;
    int64_t* d_group_base = nullptr;   // n_groups + 1
    int32_t* d_slot_id = nullptr;
    int32_t* d_slot_len = nullptr;
    int32_t* d_loc = nullptr;
    int64_t device_bytes = 0;

    DbView view() const {
        DbView v;
        v.words = d_words;
        v.group_base = d_group_base;
        v.slot_id = d_slot_id;
        v.slot_len = d_slot_len;
        v.loc = d_loc;
        v.n_groups = n_groups;
        return v;
    }
};

// One workgroup per group of 64 targets: encode letters and pack six 5-bit
// codes per word, lane-interleaved.
__global__ __launch_bounds__(256) void k_pack(const uint8_t* __restrict__ residues,
                                              const int64_t* __restrict__ offsets,
                                              const int32_t* __restrict__ slot_id,
                                              const int32_t* __restrict__ slot_len,
                                              const int64_t* __restrict__ group_base,
                                              uint32_t* __restrict__ words, int32_t* err) {
    const int32_t g = blockIdx.x;
    const int64_t base = group_base[g];
    const int64_t nw = group_base[g + 1] - base;
    for (int64_t x = threadIdx.x; x < nw; x += blockDim.x) {
        const int32_t lane = (int32_t)(x & (kLanes - 1));
        const int64_t w = x >> 6;
        const int32_t id = slot_id[g * kLanes + lane];
        uint32_t word = 0;
        if (id >= 0) {
            const int64_t len = slot_len[g * kLanes + lane];
            const uint8_t* src = residues + offsets[id];
            for (int i = 0; i < kResPerWord; ++i) {
                const int64_t p = w * kResPerWord + i;
                if (p >= len) break;
                int c = c_codes[src[p]];
                if (c < 0) {
                    atomicOr(err, 1);
                    c = 0;
                }
                word |= (uint32_t)c << (5 * i);
            }
        }
        words[base + x] = word;
    }
}

namespace {

void free_db(hs_db* db) {
    if (!db) return;
    (void)hipFree(db->d_words);
    (void)hipFree(db->d_group_base);
    (void)hipFree(db->d_slot_id);
    (void)hipFree(db->d_slot_len);
    (void)hipFree(db->d_loc);
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

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Per-query workspace carve-up.
struct QueryWs {
    int32_t* scores;
    int32_t* rounds;
    TopkState* topk;
    uint32_t* hist;
    uint64_t* keys;
};

size_t query_ws_bytes(int64_t n_targets, int32_t k) {
    return 2 * align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(n_targets, 1)) +
           align_up(sizeof(TopkState)) + align_up(sizeof(uint32_t) * kTopkBins) +
           align_up(sizeof(uint64_t) * (size_t)std::max(k, 1));
}

QueryWs carve(void* ws, int64_t n_targets, int32_t k) {
    char* p = (char*)ws;
    QueryWs q;
    q.scores = (int32_t*)p;
    p += align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(n_targets, 1));
    q.rounds = (int32_t*)p;
    p += align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(n_targets, 1));
    q.topk = (TopkState*)p;
    p += align_up(sizeof(TopkState));
    q.hist = (uint32_t*)p;
    p += align_up(sizeof(uint32_t) * kTopkBins);
    q.keys = (uint64_t*)p;
    (void)k;
    return q;
}

int32_t profile_stride(int32_t qlen) { return (qlen + 3) & ~3; }

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

int launch_score(const hs_db* db, const uint8_t* d_q, int32_t qlen, const hs_params* p,
                 hipStream_t st, int32_t* d_scores, int32_t* d_rounds, uint64_t* d_cells) {
    if (db->n_groups == 0) return HS_OK;
    const int32_t ps = profile_stride(qlen);
    const size_t lds = (size_t)kNsym * ps;
    const int wg = (db->n_groups + 3) / 4;
    if (d_cells) {
        int rc = set_lds_limit((const void*)k_score_lanes<true>, lds);
        if (rc) return rc;
        hipLaunchKernelGGL(k_score_lanes<true>, dim3(wg), dim3(256), lds, st, db->view(), d_q, qlen,
                           ps, kparams(p), kmatrix(p), d_scores, d_rounds,
                           (unsigned long long*)d_cells);
    } else {
        int rc = set_lds_limit((const void*)k_score_lanes<false>, lds);
        if (rc) return rc;
        hipLaunchKernelGGL(k_score_lanes<false>, dim3(wg), dim3(256), lds, st, db->view(), d_q, qlen,
                           ps, kparams(p), kmatrix(p), d_scores, d_rounds, nullptr);
    }
    HIP_TRY(hipGetLastError());
    return HS_OK;
}

// Queues one search.  All pointers are device pointers.
int launch_search(const hs_db* db, const uint8_t* d_q, int32_t qlen, const hs_params* p, int32_t k,
                  int32_t n_aln, hipStream_t st, void* d_ws, DevHit* d_hits, int32_t* d_n_hits,
                  DevAln* d_alns, uint32_t* d_ops, int64_t ops_stride) {
    const KParams kp = kparams(p);
    const KMatrix km = kmatrix(p);
    const int32_t ps = profile_stride(qlen);
    const size_t lds = (size_t)kNsym * ps;
    QueryWs w = carve(d_ws, db->n_targets, k);
    const int32_t n = (int32_t)db->n_targets;

    int rc0 = launch_score(db, d_q, qlen, p, st, w.scores, w.rounds, nullptr);
    if (rc0) return rc0;
    hipLaunchKernelGGL(k_topk_init, dim3(1), dim3(256), 0, st, w.topk, w.hist, k);
    const int tb = std::max(1, std::min(1024, (n + 255) / 256));
    for (int pass = 0; pass < kTopkPasses; ++pass)
        hipLaunchKernelGGL(k_topk_pass, dim3(tb), dim3(256), 0, st, w.scores, n, p->min_score,
                           w.topk, w.hist, pass);
    hipLaunchKernelGGL(k_topk_collect, dim3(tb), dim3(256), 0, st, w.scores, n, p->min_score,
                       w.topk, w.keys, k);
    hipLaunchKernelGGL(k_topk_sort, dim3(1), dim3(1024), 0, st, w.topk, w.keys, w.rounds, n, k,
                       d_hits, d_n_hits);
    HIP_TRY(hipGetLastError());
    if (n_aln > 0) {
        int rc = set_lds_limit((const void*)k_traceback, lds);
        if (rc) return rc;
        hipLaunchKernelGGL(k_traceback, dim3((n_aln + 63) / 64), dim3(64), lds, st, db->view(), d_q,
                           qlen, ps, kp, km, d_hits, d_n_hits, n_aln, (int32_t)db->n_targets,
                           d_alns, d_ops, ops_stride);
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
    for (int64_t i = 0; i < n_targets; ++i) {
        const int64_t L = offsets[i + 1] - offsets[i];
        if (L < 1 || L > HS_MAX_SEQ)
            return fail(HS_EINVAL, "target " + std::to_string(i) + " has length outside [1, HS_MAX_SEQ]");
        len[(size_t)i] = (int32_t)L;
    }
    const int64_t total = n_targets ? offsets[n_targets] - offsets[0] : 0;

    // length bins: longest first, ties by index; groups of 64
    std::vector<int32_t> order((size_t)n_targets);
    for (int64_t i = 0; i < n_targets; ++i) order[(size_t)i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return len[(size_t)a] > len[(size_t)b]; });
    const int32_t n_groups = (int32_t)((n_targets + kLanes - 1) / kLanes);
    std::vector<int32_t> slot_id((size_t)n_groups * kLanes, -1), slot_len((size_t)n_groups * kLanes, 0);
    std::vector<int32_t> loc((size_t)n_targets);
    std::vector<int64_t> gbase((size_t)n_groups + 1, 0);
    for (int64_t s = 0; s < n_targets; ++s) {
        slot_id[(size_t)s] = order[(size_t)s];
        slot_len[(size_t)s] = len[(size_t)order[(size_t)s]];
        loc[(size_t)order[(size_t)s]] = (int32_t)s;
    }
    for (int32_t g = 0; g < n_groups; ++g) {
        const int64_t maxlen = slot_len[(size_t)g * kLanes];
        gbase[(size_t)g + 1] = gbase[(size_t)g] + (maxlen + kResPerWord - 1) / kResPerWord * kLanes;
    }
    const int64_t n_words = gbase[(size_t)n_groups] + kLanes;   // one spare row for read-ahead

    hs_db* db = new hs_db();
    db->n_targets = n_targets;
    db->n_residues = total;
    db->n_groups = n_groups;
    db->n_words = n_words;
    int rc = HS_OK;
    uint8_t* d_res = nullptr;
    int64_t* d_off = nullptr;
    int32_t* d_err = nullptr;
    auto cleanup = [&](int code) {
        (void)hipFree(d_res);
        (void)hipFree(d_off);
        (void)hipFree(d_err);
        if (code != HS_OK) free_db(db);
        return code;
    };
    if ((rc = dev_alloc(&db->d_words, (size_t)n_words, &db->device_bytes)) ||
        (rc = dev_alloc(&db->d_group_base, (size_t)n_groups + 1, &db->device_bytes)) ||
        (rc = dev_alloc(&db->d_slot_id, slot_id.size(), &db->device_bytes)) ||
        (rc = dev_alloc(&db->d_slot_len, slot_len.size(), &db->device_bytes)) ||
        (rc = dev_alloc(&db->d_loc, loc.size(), &db->device_bytes)) ||
        (rc = dev_alloc(&d_res, (size_t)total, nullptr)) ||
        (rc = dev_alloc(&d_off, (size_t)n_targets + 1, nullptr)) ||
        (rc = dev_alloc(&d_err, 1, nullptr)))
        return cleanup(rc);
    auto h2d = [&](void* dst, const void* src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
    };
    std::vector<int64_t> rel((size_t)n_targets + 1);
    for (int64_t i = 0; i <= n_targets; ++i) rel[(size_t)i] = n_targets ? offsets[i] - offsets[0] : 0;
    if (h2d(db->d_group_base, gbase.data(), gbase.size() * 8) != hipSuccess ||
        h2d(db->d_slot_id, slot_id.data(), slot_id.size() * 4) != hipSuccess ||
        h2d(db->d_slot_len, slot_len.data(), slot_len.size() * 4) != hipSuccess ||
        h2d(db->d_loc, loc.data(), loc.size() * 4) != hipSuccess ||
        h2d(d_res, residues + (n_targets ? offsets[0] : 0), (size_t)total) != hipSuccess ||
        h2d(d_off, rel.data(), rel.size() * 8) != hipSuccess ||
        hipMemsetAsync(d_err, 0, sizeof(int32_t), st) != hipSuccess ||
        hipMemsetAsync(db->d_words + gbase[(size_t)n_groups], 0, kLanes * 4, st) != hipSuccess ||
        hipMemcpyToSymbolAsync(HIP_SYMBOL(c_codes), kCodes.t, 256, 0, hipMemcpyHostToDevice, st) !=
            hipSuccess)
        return cleanup(fail(HS_EDEVICE, "copy to device failed"));
    if (n_groups > 0) {
        hipLaunchKernelGGL(k_pack, dim3(n_groups), dim3(256), 0, st, d_res, d_off, db->d_slot_id,
                           db->d_slot_len, db->d_group_base, db->d_words, d_err);
        if (hipGetLastError() != hipSuccess) return cleanup(fail(HS_EDEVICE, "pack launch failed"));
    }
    int32_t err = 0;
    if (hipMemcpyAsync(&err, d_err, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return cleanup(fail(HS_EDEVICE, "database packing failed"));
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
    return (size_t)nq * query_ws_bytes(db->n_targets, k);
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
                 void* stream, int32_t* d_scores, int32_t* d_rounds, uint64_t* d_cells) {
    if (!db) return fail(HS_EINVAL, "db is NULL");
    if (qlen < 1 || qlen > HS_MAX_QUERY) return fail(HS_EINVAL, "qlen must lie in [1, HS_MAX_QUERY]");
    int rc = check_params(params);
    if (rc) return rc;
    if (!d_qcodes || !d_scores) return fail(HS_EINVAL, "NULL device pointer");
    return launch_score(db, d_qcodes, qlen, params, (hipStream_t)stream, d_scores, d_rounds,
                        d_cells);
}

const char* hs_last_error(void) { return g_err.c_str(); }

}  // extern "C"
