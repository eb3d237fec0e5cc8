// rg_api.hip -- status strings, error detail and the whole-step driver.
//
// rg_step follows the order of the per-step phases in the paper's Table 1
// (compute dt, set unew, godunov, set uold, upload) with a global time step:
// optional hash + neighbour rebuild (Sec. 2.1, 2.3), CFL dt, every level's
// hydro update from uold into unew, coarse-fine flux correction, and
// restriction from the finest level down.
#include <cstdarg>
#include <cstring>
#include <mutex>

#include "rg_internal.hpp"

namespace rg {

namespace {
thread_local std::string g_detail;
}

void set_detail(const std::string &s) { g_detail = s; }

rg_status fail(rg_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_detail = std::string(rg_status_string(st)) + ": " + buf;
    return st;
}

rg_status launch_status(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RG_EHIP, "%s: %s", what, hipGetErrorString(e));
    return RG_OK;
}

// ---------------------------------------------------------------------------
// device-side error sink of calls that have no hash workspace
// ---------------------------------------------------------------------------

namespace {
// one per device; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device
__device__ HashHeader g_err_sink;

constexpr int kMaxDevices = 64;
std::mutex g_sink_mu;
HashHeader *g_sink_addr[kMaxDevices] = {};
thread_local HashHeader *tl_sink = nullptr;
}  // namespace

HashHeader *err_sink()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_sink_mu);
    if (!g_sink_addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_err_sink)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_sink_addr[dev] = static_cast<HashHeader *>(p);
    }
    return g_sink_addr[dev];
}

HashHeader *current_sink() { return tl_sink ? tl_sink : err_sink(); }

SinkScope::SinkScope(void *d_hash_ws) : prev(tl_sink)
{
    if (d_hash_ws) tl_sink = static_cast<HashHeader *>(d_hash_ws);
}

SinkScope::~SinkScope() { tl_sink = prev; }

// reads and clears the library's own error word (rg_check with no workspace)
rg_status check_sink(int64_t *h_bad_index, hipStream_t s)
{
    HashHeader *d = err_sink();
    if (!d) return fail(RG_EHIP, "rg_check: no error word on this device");
    HashHeader h;
    hipError_t e = hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(RG_EHIP, "rg_check: %s", hipGetErrorString(e));
    if (h.err) {
        HashHeader z;
        memset(&z, 0, sizeof(z));
        e = hipMemcpyAsync(d, &z, sizeof(z), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return fail(RG_EHIP, "rg_check: %s", hipGetErrorString(e));
    }
    if (h_bad_index) *h_bad_index = h.err ? h.bad : -1;
    if (h.err) return fail(static_cast<rg_status>(h.err), "device reported %s at index %lld",
                           rg_status_string(h.err), static_cast<long long>(h.bad));
    return RG_OK;
}

struct LevelArgs;
rg_status hydro_level(const LevelArgs &a, int form, const rg_tuning *tune, hipStream_t s);
rg_status coarse_corrections_list(double *unew, const double *corr, int64_t corr_base, const int32_t *nbr27,
                                  const int32_t *list, int64_t count, hipStream_t s);

}  // namespace rg

using namespace rg;

extern "C" {

int rg_abi_version(void) { return RG_ABI_VERSION; }

const char *rg_status_string(int status)
{
    switch (status) {
    case RG_OK: return "RG_OK";
    case RG_EINVAL: return "RG_EINVAL";
    case RG_EFULL: return "RG_EFULL";
    case RG_EDUPKEY: return "RG_EDUPKEY";
    case RG_EUNGRADED: return "RG_EUNGRADED";
    case RG_ENONFINITE: return "RG_ENONFINITE";
    case RG_EHIP: return "RG_EHIP";
    case RG_ENOTSUP: return "RG_ENOTSUP";
    default: return "RG_UNKNOWN";
    }
}

size_t rg_last_error_detail(char *buf, size_t len)
{
    if (buf && len) {
        size_t n = g_detail.size() < len - 1 ? g_detail.size() : len - 1;
        memcpy(buf, g_detail.data(), n);
        buf[n] = '\0';
    }
    return g_detail.size();
}

rg_status rg_prepare_tree(const rg_tree *t, unsigned flags, void *stream)
{
    RG_REQUIRE(t && t->n_oct > 0, "bad tree");
    RG_REQUIRE((flags & ~(RG_STEP_REBUILD | RG_STEP_REKEY)) == 0, "unknown flags %u", flags);
    if (flags & RG_STEP_REKEY) {
        RG_REQUIRE(t->d_ijkl && t->d_keys_scratch && t->d_perm && t->d_sort_ws && t->d_level_begin,
                   "RG_STEP_REKEY needs coordinates, scratch keys, permutation, sort workspace and level ranges");
        RG_TRY(rg_encode_keys(t->d_ijkl, t->n_oct, t->d_keys_scratch, stream));
        RG_TRY(sort_keys_bits(t->d_keys_scratch, t->n_oct, t->d_keys, t->d_perm, t->d_sort_ws, t->sort_ws_bytes,
                              3 * t->lmax, as_stream(stream)));
        RG_TRY(rg_level_ranges(t->d_keys, t->n_oct, t->d_level_begin, stream));
    }
    if (flags & RG_STEP_REBUILD) {
        RG_TRY(rg_hash_build(t->d_keys, t->n_oct, t->d_hash_ws, t->hash_ws_bytes, stream));
        if (t->sched && t->sched->d_list) {
            const rg_schedule *sc = t->sched;
            RG_TRY(neighbours_scheduled(t->d_hash_ws, t->d_keys, t->n_oct, t->lmin, t->lmax,
                                        t->level_begin[t->lmax], t->bc,
                                        sc->d_list + sc->nbr_brick_begin, sc->nbr_brick_count,
                                        sc->d_list + sc->nbr_rest_begin, sc->nbr_rest_count, t->d_nbr27,
                                        t->d_father_cell, t->d_son_mask, as_stream(stream)));
        } else {
            RG_TRY(rg_build_neighbours(t->d_hash_ws, t->d_keys, t->n_oct, t->lmin, t->bc, t->d_nbr27,
                                       t->d_father_cell, t->d_son_mask, stream));
        }
    }
    return RG_OK;
}

rg_status rg_step(const rg_tree *t, const double *d_uold, double *d_unew, double gamma, double cfl, int form,
                  unsigned flags, double *d_dt, const rg_tuning *tune, void *stream)
{
    RG_REQUIRE(t && d_uold && d_unew && d_dt, "null pointer");
    RG_REQUIRE(t->n_oct > 0 && t->lmin >= 1 && t->lmax >= t->lmin && t->lmax <= RG_MAX_LEVEL, "bad tree");
    RG_REQUIRE(t->level_begin[t->lmin] == 0 && t->level_begin[t->lmax + 1] == t->n_oct, "bad level ranges");
    RG_REQUIRE(t->lmin == t->lmax || t->d_corr, "a multilevel tree needs a correction buffer");
    RG_REQUIRE((flags & ~(RG_STEP_REBUILD | RG_STEP_REKEY | RG_STEP_CHAIN_DT)) == 0, "unknown flags %u", flags);
    RG_REQUIRE(gamma > 1 && cfl > 0, "bad gamma or cfl");
    RG_REQUIRE(t->ghost == RG_GHOST_INJECT || t->ghost == RG_GHOST_LINEAR, "bad ghost mode %d", t->ghost);
    hipStream_t s = as_stream(stream);
    const SinkScope sink(t->d_hash_ws);
    const unsigned prep = flags & (RG_STEP_REBUILD | RG_STEP_REKEY);
    if (prep) RG_TRY(rg_prepare_tree(t, prep, stream));
    const bool chain = (flags & RG_STEP_CHAIN_DT) != 0;
    double *dt_next = chain ? d_dt + 1 : nullptr;
    if (chain) {
        RG_TRY(set_u64(reinterpret_cast<uint64_t *>(dt_next), 0x7ff0000000000000ull, s));
    } else {
        RG_TRY(rg_cfl_dt(d_uold, t->d_son_mask, t->level_begin, t->lmin, t->lmax, gamma, cfl, d_dt, stream));
    }
    const int64_t corr_base = t->level_begin[t->lmin + 1];
    for (int l = t->lmin; l <= t->lmax; ++l) {
        const int64_t b = t->level_begin[l], e = t->level_begin[l + 1];
        if (e == b) continue;
        if (t->sched) {
            RG_TRY(rg_hydro_step_scheduled(t, t->sched, l, d_dt, gamma, d_uold, d_unew, cfl, dt_next, form, tune,
                                           stream));
        } else {
            RG_TRY(rg_hydro_step_level(ldexp(1.0, -l), d_dt, gamma, d_uold, d_unew, t->d_nbr27, t->d_son_mask, b, e,
                                       l > t->lmin ? t->d_corr : nullptr, corr_base, cfl, dt_next, form, tune,
                                       stream));
        }
    }
    if (t->lmax > t->lmin) {
        if (t->sched) {
            // the border lists of all levels above lmin follow each other
            const rg_schedule *sc = t->sched;
            const int64_t b = sc->border_begin[t->lmin + 1];
            const int64_t e = sc->border_begin[t->lmax] + sc->border_count[t->lmax];
            RG_TRY(coarse_corrections_list(d_unew, t->d_corr, corr_base, t->d_nbr27, sc->d_list + b, e - b, s));
        } else {
            RG_TRY(rg_apply_coarse_corrections(d_unew, t->d_corr, corr_base, t->d_nbr27, corr_base, t->n_oct, stream));
        }
        if (chain)
            RG_TRY(rg_cfl_dt_corrected(d_unew, t->d_nbr27, t->level_begin, t->lmin, t->lmax, gamma, cfl, dt_next,
                                       stream));
        for (int l = t->lmax; l > t->lmin; --l)
            RG_TRY(rg_restrict_level(d_unew, t->d_father_cell, t->level_begin[l], t->level_begin[l + 1], stream));
    }
    return RG_OK;
}

}  // extern "C"
