// C ABI of the rDDMC library: argument validation, table/tally layout, host staging of
// the small per-cloud inputs, and kernel launches.  No transport arithmetic runs here.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <climits>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "rddmc_internal.h"
#include "surrogate_dev.h"

using namespace rddmc;

namespace {

thread_local std::string g_err;

rddmc_status fail(rddmc_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

rddmc_status hip_fail(hipError_t e, const char *what)
{
    return fail(RDDMC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

bool finite_all(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

bool increasing(const double *p, size_t n)
{
    for (size_t i = 0; i + 1 < n; ++i)
        if (!(p[i] < p[i + 1])) return false;
    return true;
}

// Emission states of one source coordinate: the containing cell, or both cells (1/2
// each) when the coordinate lies exactly on an interior face.
bool split_coord(const double *f, int n, double v, std::vector<std::pair<int, double>> &out)
{
    out.clear();
    if (!(v >= f[0] && v <= f[n])) return false;
    for (int e = 0; e <= n; ++e) {
        if (f[e] == v) {
            if (e == 0) out.push_back({0, 1.0});
            else if (e == n) out.push_back({n - 1, 1.0});
            else {
                out.push_back({e - 1, 0.5});
                out.push_back({e, 0.5});
            }
            return true;
        }
    }
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (v >= f[mid]) lo = mid; else hi = mid;
    }
    out.push_back({lo, 1.0});
    return true;
}

struct Layout {
    DevHeader h{};
    std::vector<DevCloud> clouds;
    std::vector<uint64_t> prefix;
    std::vector<std::vector<int32_t>> src_state;
    std::vector<std::vector<double>> src_cdf;
    std::vector<std::vector<float>> src_pos;     // 3D: {x, y, z, frequency} per emission entry
    std::vector<std::vector<double>> src_t;      // hybrid 1D: emission window per entry
    uint64_t table_bytes = 0;
    uint64_t tally_words = 0;
    bool any_moving = false;
};

rddmc_status validate_cloud(const rddmc_medium &m, int idx)
{
    if (m.geometry != RDDMC_SLAB && m.geometry != RDDMC_SPHERE && m.geometry != RDDMC_CART3D)
        return fail(RDDMC_EINVAL, "cloud %d: unknown geometry %d", idx, m.geometry);
    const int nd = m.geometry == RDDMC_CART3D ? 3 : 1;
    for (int d = 0; d < 3; ++d) {
        if (m.n_cells[d] < 1) return fail(RDDMC_EINVAL, "cloud %d: n_cells[%d] < 1", idx, d);
        if (d >= nd && m.n_cells[d] != 1)
            return fail(RDDMC_EINVAL, "cloud %d: 1D geometry needs n_cells = {n,1,1}", idx);
    }
    if (m.n_bins < 1) return fail(RDDMC_EINVAL, "cloud %d: n_bins < 1", idx);
    for (int d = 0; d < nd; ++d) {
        if (!m.faces[d]) return fail(RDDMC_EINVAL, "cloud %d: faces[%d] is NULL", idx, d);
        if (!finite_all(m.faces[d], m.n_cells[d] + 1) || !increasing(m.faces[d], m.n_cells[d] + 1))
            return fail(RDDMC_EINVAL, "cloud %d: faces[%d] not finite and strictly increasing", idx, d);
    }
    if (m.geometry == RDDMC_SPHERE && m.faces[0][0] < 0.0)
        return fail(RDDMC_EINVAL, "cloud %d: negative sphere radius", idx);
    if (!m.bin_edges || !finite_all(m.bin_edges, m.n_bins + 1) || !increasing(m.bin_edges, m.n_bins + 1))
        return fail(RDDMC_EINVAL, "cloud %d: bin edges not finite and strictly increasing", idx);
    const int64_t nc = (int64_t)m.n_cells[0] * m.n_cells[1] * m.n_cells[2];
    if (!m.k0 || !m.temp) return fail(RDDMC_EINVAL, "cloud %d: k0/temp NULL", idx);
    for (int64_t c = 0; c < nc; ++c) {
        if (!(m.k0[c] > 0.0) || !std::isfinite(m.k0[c]))
            return fail(RDDMC_EINVAL, "cloud %d: k0[%lld] must be finite and > 0", idx, (long long)c);
        if (!(m.temp[c] > 0.0) || !std::isfinite(m.temp[c]))
            return fail(RDDMC_EINVAL, "cloud %d: temp[%lld] must be finite and > 0", idx, (long long)c);
    }
    if (m.vel && !finite_all(m.vel, (size_t)nc * (m.geometry == RDDMC_CART3D ? 3 : 1)))
        return fail(RDDMC_EINVAL, "cloud %d: non-finite velocity", idx);
    if (!(m.tau_threshold == 0.0 || m.tau_threshold >= 2.0) || !std::isfinite(m.tau_threshold))
        return fail(RDDMC_EINVAL, "cloud %d: tau_threshold must be 0 (pure DDMC) or >= 2", idx);
    if (!(m.f_mu >= 0.0 && m.f_mu <= 1.0)) return fail(RDDMC_EINVAL, "cloud %d: f_mu outside [0,1]", idx);
    if (!(m.lambda > 0.0) || !std::isfinite(m.lambda)) return fail(RDDMC_EINVAL, "cloud %d: lambda <= 0", idx);
    if (m.n_src < 1 || !m.src_pos || !m.src_x) return fail(RDDMC_EINVAL, "cloud %d: no sources", idx);
    if (m.n_packets >= (1ull << 32)) return fail(RDDMC_EINVAL, "cloud %d: n_packets >= 2^32", idx);
    if (!(m.x_crit >= 0.0) || !std::isfinite(m.x_crit))
        return fail(RDDMC_EINVAL, "cloud %d: x_crit must be finite and >= 0", idx);
    for (const double *d : {m.dust_abs, m.dust_sca})
        if (d)
            for (int64_t c = 0; c < nc; ++c)
                if (!(d[c] >= 0.0) || !std::isfinite(d[c]))
                    return fail(RDDMC_EINVAL, "cloud %d: dust coefficients must be finite and >= 0", idx);
    if (m.src_t)
        for (int s = 0; s < m.n_src; ++s) {
            const double a = m.src_t[2 * s], b = m.src_t[2 * s + 1];
            if (!(a >= 0.0) || !(b >= a) || !std::isfinite(b))
                return fail(RDDMC_EINVAL, "cloud %d: emission window %d must satisfy 0 <= t_start <= t_end", idx, s);
        }
    if (m.n_census < 0 || m.n_census > 4096 || (m.n_census > 0) != (m.census != nullptr))
        return fail(RDDMC_EINVAL, "cloud %d: n_census in [0, 4096] with census given iff n_census > 0", idx);
    if (m.n_census > 0 && (!finite_all(m.census, m.n_census + 1) || !increasing(m.census, m.n_census + 1) ||
                           m.census[0] < 0.0))
        return fail(RDDMC_EINVAL, "cloud %d: census times must be finite, >= 0 and increasing", idx);
    const bool extras = m.dust_abs || m.dust_sca || m.src_t || m.n_census > 0;
    if (extras && m.geometry == RDDMC_CART3D)
        return fail(RDDMC_EUNSUPPORTED, "cloud %d: dust, emission windows and census tallies are for 1D clouds", idx);
    if ((m.flags & RDDMC_FLAG_DUST_WEIGHT) && !m.dust_abs)
        return fail(RDDMC_EINVAL, "cloud %d: RDDMC_FLAG_DUST_WEIGHT needs dust_abs", idx);
    if (m.flags & RDDMC_FLAG_GROUPS) {   // frequency groups (Sec. 5.3): one table per cloud
        if (m.geometry == RDDMC_CART3D)
            return fail(RDDMC_EUNSUPPORTED, "cloud %d: frequency groups are for 1D clouds", idx);
        if (m.vel)
            for (int64_t c = 0; c < nc; ++c)
                if (m.vel[c] != 0.0) return fail(RDDMC_EUNSUPPORTED, "cloud %d: frequency groups need a static medium", idx);
        for (int64_t c = 1; c < nc; ++c)
            if (m.temp[c] != m.temp[0])
                return fail(RDDMC_EUNSUPPORTED, "cloud %d: frequency groups need one temperature for all cells", idx);
        if (!(m.tau_threshold > 0.0))
            return fail(RDDMC_EINVAL, "cloud %d: frequency groups need continuous-MC states (tau_threshold > 0)", idx);
        if (m.x_crit != 0.0) return fail(RDDMC_EINVAL, "cloud %d: core-skipping does not apply to frequency groups", idx);
        if (m.n_bins > RDDMC_MAX_GROUP_BINS)
            return fail(RDDMC_EINVAL, "cloud %d: frequency groups take at most %d bins", idx, RDDMC_MAX_GROUP_BINS);
    }
    return RDDMC_OK;
}

rddmc_status make_layout(const rddmc_batch *b, Layout &L)
{
    if (!b || b->n_clouds < 1 || !b->clouds) return fail(RDDMC_EINVAL, "empty batch");
    const int n = b->n_clouds;
    L.clouds.assign(n, DevCloud{});
    L.prefix.assign(n + 1, 0);
    L.src_state.assign(n, {});
    L.src_cdf.assign(n, {});
    L.src_pos.assign(n, {});
    L.src_t.assign(n, {});
    const int geom = b->clouds[0].geometry;
    // a 1D batch with a continuous-MC option (tau_threshold > 0 or core-skipping) is walked by
    // the hybrid 1D walk: flag layout, MC cell records and line tables for every cloud
    bool hybrid1d = false;
    if (geom != RDDMC_CART3D)
        for (int ci = 0; ci < n; ++ci) {
            const rddmc_medium &m = b->clouds[ci];
            hybrid1d |= m.tau_threshold > 0.0 || m.x_crit > 0.0 || m.dust_abs || m.dust_sca || m.src_t ||
                        m.n_census > 0;
        }
    const bool flagged = geom == RDDMC_CART3D || hybrid1d;
    uint64_t off = 0;
    L.h.n_clouds = n;
    L.h.geometry = geom;
    L.h.hybrid1d = hybrid1d ? 1u : 0u;
    off = align_up(sizeof(DevHeader));
    L.h.off_clouds = off;
    off = align_up(off + sizeof(DevCloud) * n);
    L.h.off_prefix = off;
    off = align_up(off + sizeof(uint64_t) * (n + 1));
    if (flagged) {   // FP32 line tables of the continuous-MC step
        L.h.off_voigt = off;
        off = align_up(off + 4ull * kVoigtN);
        L.h.off_u0 = off;
        off = align_up(off + 4ull * kU0NA * kU0NX);
    }
    uint64_t tally = 0;
    for (int ci = 0; ci < n; ++ci) {
        const rddmc_medium &m = b->clouds[ci];
        rddmc_status st = validate_cloud(m, ci);
        if (st != RDDMC_OK) return st;
        if (m.geometry != geom) return fail(RDDMC_EUNSUPPORTED, "mixed geometries in one batch");
        DevCloud &c = L.clouds[ci];
        c.geometry = m.geometry;
        c.nb = m.n_bins;
        c.n[0] = m.n_cells[0];
        c.n[1] = m.n_cells[1];
        c.n[2] = m.n_cells[2];
        c.nc = m.n_cells[0] * m.n_cells[1] * m.n_cells[2];
        c.nf = m.geometry == RDDMC_CART3D ? 6 : 2;
        c.n_rows = m.geometry == RDDMC_SLAB ? 2 : (m.geometry == RDDMC_SPHERE ? 1 : 6);
        c.keep_rates = (m.flags & RDDMC_FLAG_KEEP_RATES) ? 1 : 0;
        c.dirichlet = (m.flags & RDDMC_FLAG_DIRICHLET) ? 1 : 0;
        c.moving = 0;
        if (m.vel) {
            const size_t nv = (size_t)c.nc * (m.geometry == RDDMC_CART3D ? 3 : 1);
            for (size_t i = 0; i < nv; ++i)
                if (m.vel[i] != 0.0) c.moving = 1;
        }
        L.any_moving |= c.moving != 0;
        c.n_packets = m.n_packets;
        c.stream = m.stream;
        c.packet_base = L.prefix[ci];
        L.prefix[ci + 1] = L.prefix[ci] + m.n_packets;
        c.n_states = (uint64_t)c.nc * c.nb;
        c.tau_th = m.tau_threshold;
        {
            const double e0 = m.bin_edges[0], dxu = (m.bin_edges[m.n_bins] - e0) / m.n_bins;
            bool uni = true;
            for (int j = 0; j <= m.n_bins && uni; ++j)
                uni = std::fabs(m.bin_edges[j] - (e0 + j * dxu)) <= 1e-9 * std::fabs(dxu);
            c.uniform_bins = uni ? 1 : 0;
            c.x0 = (float)e0;
            c.dx = (float)dxu;
            c.inv_dx = (float)(1.0 / dxu);
        }
        c.f_mu = m.f_mu;
        c.lambda = m.lambda;
        c.flag_layout = flagged ? 1 : 0;
        c.x_crit = (float)m.x_crit;
        c.dusty = (m.dust_abs || m.dust_sca) ? 1 : 0;
        c.n_census = m.n_census;
        // sources -> (state, probability); 3D keeps one entry per (source, state) with the
        // source's position and frequency (a packet starting in a thin state needs them)
        std::map<int32_t, double> acc;
        std::vector<std::pair<int, double>> bins, cx, cy, cz;
        double cum3 = 0.0;
        for (int s = 0; s < m.n_src; ++s) {
            if (!split_coord(m.bin_edges, m.n_bins, m.src_x[s], bins))
                return fail(RDDMC_EINVAL, "cloud %d: source %d frequency outside the grid", ci, s);
            const double *p = m.src_pos + 3 * s;
            if (!split_coord(m.faces[0], m.n_cells[0], p[0], cx))
                return fail(RDDMC_EINVAL, "cloud %d: source %d outside the grid", ci, s);
            if (m.geometry != RDDMC_CART3D && !hybrid1d) {
                for (auto &a : cx)
                    for (auto &bb : bins)
                        acc[a.first * m.n_bins + bb.first] += a.second * bb.second / m.n_src;
                continue;
            }
            if (m.geometry != RDDMC_CART3D) {   // hybrid 1D: one entry per (source, state)
                for (auto &a : cx)
                    for (auto &bb : bins) {
                        cum3 += a.second * bb.second / m.n_src;
                        L.src_state[ci].push_back((int32_t)(a.first * m.n_bins + bb.first));
                        L.src_cdf[ci].push_back(cum3);
                        L.src_pos[ci].push_back(0.0f);
                        L.src_pos[ci].push_back(0.0f);
                        L.src_pos[ci].push_back((float)p[0]);
                        L.src_pos[ci].push_back((float)m.src_x[s]);
                        L.src_t[ci].push_back(m.src_t ? m.src_t[2 * s] : 0.0);
                        L.src_t[ci].push_back(m.src_t ? m.src_t[2 * s + 1] : 0.0);
                    }
                continue;
            }
            if (!split_coord(m.faces[1], m.n_cells[1], p[1], cy) || !split_coord(m.faces[2], m.n_cells[2], p[2], cz))
                return fail(RDDMC_EINVAL, "cloud %d: source %d outside the grid", ci, s);
            for (auto &ax : cx)
                for (auto &ay : cy)
                    for (auto &az : cz)
                        for (auto &bb : bins) {
                            const int64_t cell = ((int64_t)az.first * m.n_cells[1] + ay.first) * m.n_cells[0] + ax.first;
                            const int64_t st = cell * m.n_bins + bb.first;
                            if (st > INT32_MAX) return fail(RDDMC_ESIZE, "cloud %d: source state index >= 2^31", ci);
                            cum3 += ax.second * ay.second * az.second * bb.second / m.n_src;
                            L.src_state[ci].push_back((int32_t)st);
                            L.src_cdf[ci].push_back(cum3);
                            for (int d = 0; d < 3; ++d) L.src_pos[ci].push_back((float)p[d]);
                            L.src_pos[ci].push_back((float)m.src_x[s]);
                        }
        }
        if (m.geometry != RDDMC_CART3D && !hybrid1d) {
            double cum = 0.0;
            for (auto &kv : acc) {
                cum += kv.second;
                L.src_state[ci].push_back(kv.first);
                L.src_cdf[ci].push_back(cum);
            }
        }
        L.src_cdf[ci].back() = 1.0;
        c.n_src = (int32_t)L.src_state[ci].size();
        // table regions
        auto take = [&](uint64_t bytes) {
            const uint64_t o = off;
            off = align_up(off + bytes);
            return o;
        };
        c.off_edges = take(8ull * (c.nb + 1));
        for (int d = 0; d < 3; ++d) c.off_faces[d] = take(8ull * (c.n[d] + 1));
        c.off_k0 = take(8ull * c.nc);
        c.off_T = take(8ull * c.nc);
        c.off_vel = take(8ull * c.nc * (m.geometry == RDDMC_CART3D ? 3 : 1));
        c.off_src_state = take(4ull * c.n_src);
        c.off_src_cdf = take(8ull * c.n_src);
        c.off_src_pos = take(16ull * c.n_src);
        c.off_k = take(8ull * c.n_states);
        c.off_hot = take(sizeof(HotRecord) * c.n_states);
        c.off_lo_words = take(16ull * c.n_states);
        c.off_face_split = take(4ull * c.n_states * (c.nf - 1));
        c.off_rates = c.keep_rates ? take(8ull * c.n_states * (c.nf + 2)) : 0;
        c.off_map = take(8ull * 3 * c.nc * c.nf);
        c.off_cmap = take(16ull * c.nc);
        c.off_mcell = flagged ? take(32ull * c.nc) : 0;
        c.off_dust = c.dusty ? take(16ull * c.nc) : 0;
        c.off_src_t = hybrid1d ? take(16ull * c.n_src) : 0;
        c.off_census = c.n_census > 0 ? take(8ull * (c.n_census + 1)) : 0;
        c.groups = (m.flags & RDDMC_FLAG_GROUPS) ? 1 : 0;
        c.dust_weight = (m.flags & RDDMC_FLAG_DUST_WEIGHT) ? 1 : 0;
        if (c.dust_weight) L.h.dust_weight1d = 1u;
        if (m.n_census > 0) L.h.census1d = 1u;
        c.off_grp_prob = c.groups ? take(8ull * c.nb * c.nb) : 0;
        c.off_grp_alias = c.groups ? take(8ull * c.nb * c.nb) : 0;
        c.n_pix = m.geometry == RDDMC_CART3D
                      ? 2ull * ((uint64_t)c.n[1] * c.n[2] + (uint64_t)c.n[0] * c.n[2] + (uint64_t)c.n[0] * c.n[1])
                      : 0;
        c.tally_off = tally;
        c.tally_words = kTallyHeader + (uint64_t)c.n_rows * (c.nb + 2) + (RDDMC_TIME_BINS + 2) + RDDMC_STEP_BINS +
                        c.n_pix;
        if (c.n_census > 0) {
            c.census_bin_off = c.tally_words;
            c.census_path_off = c.census_bin_off + (uint64_t)(c.n_census + 1) * c.n_states;
            c.census_accel_off = c.census_path_off + (uint64_t)c.n_census * c.n_states;
            c.tally_words = c.census_accel_off + (uint64_t)c.n_census * c.nc;
        }
        if (c.dust_weight) {
            c.wspec_off = c.tally_words;
            c.tally_words += 4 + 2ull * c.n_rows * (c.nb + 2);
        }
        tally += c.tally_words;
    }
    L.h.total_packets = L.prefix[n];
    L.table_bytes = off;
    L.tally_words = tally;
    return RDDMC_OK;
}

void put(std::vector<uint8_t> &buf, uint64_t off, const void *src, size_t bytes)
{
    if (bytes) std::memcpy(buf.data() + off, src, bytes);
}

}  // namespace

// Work area of rddmc_transport_static: queue counters and the cooperative tail walk's export
// slots, in device memory the library owns (one copy per device, held until the process
// ends).  Host code never passes this name to a kernel: it is a host-side stand-in, and the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned long long scratch[RDDMC_STATIC_WORK_BYTES / 8];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the calling thread's current device.
rddmc_status static_work_of_current_device(void **ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(RDDMC_EUNSUPPORTED, "device index %d >= %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(RDDMC_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return RDDMC_OK;
}

}  // namespace

extern "C" {

int32_t rddmc_abi_version(void) { return RDDMC_ABI_VERSION; }

const char *rddmc_last_error(void) { return g_err.c_str(); }

rddmc_status rddmc_table_bytes(const rddmc_batch *batch, size_t *bytes)
{
    if (!bytes) return fail(RDDMC_EINVAL, "bytes is NULL");
    Layout L;
    rddmc_status st = make_layout(batch, L);
    if (st != RDDMC_OK) return st;
    *bytes = L.table_bytes;
    return RDDMC_OK;
}

rddmc_status rddmc_tally_bytes(const rddmc_batch *batch, size_t *bytes)
{
    if (!bytes) return fail(RDDMC_EINVAL, "bytes is NULL");
    Layout L;
    rddmc_status st = make_layout(batch, L);
    if (st != RDDMC_OK) return st;
    *bytes = L.tally_words * 8;
    return RDDMC_OK;
}

rddmc_status rddmc_work_bytes(const rddmc_batch *batch, size_t *bytes)
{
    if (!bytes) return fail(RDDMC_EINVAL, "bytes is NULL");
    Layout L;
    rddmc_status st = make_layout(batch, L);
    if (st != RDDMC_OK) return st;
    // queue counters, then one 48-byte slot per lane that may hand its packet to the
    // cooperative tail walk (at most 2^20 lanes are ever resident)
    const uint64_t lanes = L.h.total_packets < (1ull << 20) ? L.h.total_packets : (1ull << 20);
    *bytes = 256 + 48 * lanes;
    return RDDMC_OK;
}

rddmc_status rddmc_build_leakage(const rddmc_batch *batch, void *d_tables, size_t table_bytes, void *stream)
{
    Layout L;
    rddmc_status st = make_layout(batch, L);
    if (st != RDDMC_OK) return st;
    if (!d_tables) return fail(RDDMC_EINVAL, "d_tables is NULL");
    if ((uintptr_t)d_tables % kAlign) return fail(RDDMC_EINVAL, "d_tables must be 256-byte aligned");
    if (table_bytes < L.table_bytes)
        return fail(RDDMC_ESIZE, "table buffer %zu < required %llu", table_bytes, (unsigned long long)L.table_bytes);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // Stage the header, descriptors and prefix, then each cloud's input copies (a
    // contiguous region per cloud).  Derived arrays are written by the kernels.
    hipError_t e;
    std::vector<std::vector<uint8_t>> bufs;
    {
        const uint64_t hdr_end = L.clouds[0].off_edges;
        bufs.emplace_back(hdr_end, 0);
        auto &buf = bufs.back();
        put(buf, 0, &L.h, sizeof L.h);
        put(buf, L.h.off_clouds, L.clouds.data(), sizeof(DevCloud) * L.clouds.size());
        put(buf, L.h.off_prefix, L.prefix.data(), 8 * L.prefix.size());
        if ((e = hipMemcpyAsync(d_tables, buf.data(), hdr_end, hipMemcpyHostToDevice, s)) != hipSuccess)
            return hip_fail(e, "hipMemcpyAsync(header)");
    }
    for (int ci = 0; ci < L.h.n_clouds; ++ci) {
        const rddmc_medium &m = batch->clouds[ci];
        const DevCloud &c = L.clouds[ci];
        const uint64_t a = c.off_edges, z = c.off_src_pos + 16ull * c.n_src;
        // regions after the input block, staged separately
        bufs.emplace_back(z - a, 0);
        auto &buf = bufs.back();
        put(buf, c.off_edges - a, m.bin_edges, 8ull * (c.nb + 1));
        for (int d = 0; d < 3; ++d) {
            if (m.faces[d] && (d == 0 || c.geometry == RDDMC_CART3D)) {
                put(buf, c.off_faces[d] - a, m.faces[d], 8ull * (c.n[d] + 1));
            } else {
                const double unit[2] = {0.0, 1.0};
                put(buf, c.off_faces[d] - a, unit, 16);
            }
        }
        put(buf, c.off_k0 - a, m.k0, 8ull * c.nc);
        put(buf, c.off_T - a, m.temp, 8ull * c.nc);
        if (m.vel) put(buf, c.off_vel - a, m.vel, 8ull * c.nc * (c.geometry == RDDMC_CART3D ? 3 : 1));
        put(buf, c.off_src_state - a, L.src_state[ci].data(), 4ull * c.n_src);
        put(buf, c.off_src_cdf - a, L.src_cdf[ci].data(), 8ull * c.n_src);
        if (c.flag_layout) put(buf, c.off_src_pos - a, L.src_pos[ci].data(), 16ull * c.n_src);
        if ((e = hipMemcpyAsync(static_cast<uint8_t *>(d_tables) + a, buf.data(), z - a, hipMemcpyHostToDevice,
                                s)) != hipSuccess)
            return hip_fail(e, "hipMemcpyAsync(inputs)");
        // dust coefficients, emission windows and census times (small per-cloud arrays)
        if (c.off_dust) {
            bufs.emplace_back(16ull * c.nc, 0);
            auto &d = bufs.back();
            for (int64_t i = 0; i < c.nc; ++i) {
                const double ka = m.dust_abs ? m.dust_abs[i] : 0.0, ks = m.dust_sca ? m.dust_sca[i] : 0.0;
                put(d, 16ull * i, &ka, 8);
                put(d, 16ull * i + 8, &ks, 8);
            }
            if ((e = hipMemcpyAsync(static_cast<uint8_t *>(d_tables) + c.off_dust, d.data(), d.size(),
                                    hipMemcpyHostToDevice, s)) != hipSuccess)
                return hip_fail(e, "hipMemcpyAsync(dust)");
        }
        if (c.off_src_t) {
            bufs.emplace_back(16ull * c.n_src, 0);
            put(bufs.back(), 0, L.src_t[ci].data(), 16ull * c.n_src);
            if ((e = hipMemcpyAsync(static_cast<uint8_t *>(d_tables) + c.off_src_t, bufs.back().data(),
                                    16ull * c.n_src, hipMemcpyHostToDevice, s)) != hipSuccess)
                return hip_fail(e, "hipMemcpyAsync(emission windows)");
        }
        if (c.off_census) {
            bufs.emplace_back(8ull * (c.n_census + 1), 0);
            put(bufs.back(), 0, m.census, 8ull * (c.n_census + 1));
            if ((e = hipMemcpyAsync(static_cast<uint8_t *>(d_tables) + c.off_census, bufs.back().data(),
                                    8ull * (c.n_census + 1), hipMemcpyHostToDevice, s)) != hipSuccess)
                return hip_fail(e, "hipMemcpyAsync(census)");
        }
    }
    for (int ci = 0; ci < L.h.n_clouds; ++ci) {
        if ((e = launch_build(L.clouds[ci], ci, static_cast<uint8_t *>(d_tables), s)) != hipSuccess)
            return hip_fail(e, "build kernels");
        if ((e = launch_build_redistribution(L.clouds[ci], static_cast<uint8_t *>(d_tables), s)) != hipSuccess)
            return hip_fail(e, "redistribution kernels");
    }
    if ((e = launch_build_line_tables(L.h, static_cast<uint8_t *>(d_tables), s)) != hipSuccess)
        return hip_fail(e, "line-table kernels");
    uint32_t flags = 0;
    if ((e = hipMemcpyAsync(&flags, &reinterpret_cast<DevHeader *>(d_tables)->error_flags, 4,
                            hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(flags)");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (flags & BE_NONFINITE) return fail(RDDMC_ENUMERIC, "a leakage table entry is non-finite or non-positive");
    if (flags & BE_THIN) return fail(RDDMC_ENUMERIC, "a thin state in a cloud without continuous-MC states");
    return RDDMC_OK;
}

rddmc_status rddmc_tally_reset(const rddmc_batch *batch, void *d_tally, size_t tally_bytes, void *stream)
{
    Layout L;
    rddmc_status st = make_layout(batch, L);
    if (st != RDDMC_OK) return st;
    if (!d_tally) return fail(RDDMC_EINVAL, "d_tally is NULL");
    if (tally_bytes < L.tally_words * 8) return fail(RDDMC_ESIZE, "tally buffer too small");
    hipError_t e = launch_zero(d_tally, L.tally_words, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? RDDMC_OK : hip_fail(e, "zero kernel");
}

rddmc_status rddmc_transport(const rddmc_batch *batch, const void *d_tables, const rddmc_run *run,
                             void *d_tally, size_t tally_bytes, void *d_work, size_t work_bytes, void *stream)
{
    Layout L;
    rddmc_status st = make_layout(batch, L);
    if (st != RDDMC_OK) return st;
    if (!d_tables || !run || !d_tally || !d_work) return fail(RDDMC_EINVAL, "NULL argument");
    if (tally_bytes < L.tally_words * 8) return fail(RDDMC_ESIZE, "tally buffer too small");
    if (work_bytes < 256) return fail(RDDMC_ESIZE, "work buffer too small");
    if (run->max_steps < 1) return fail(RDDMC_EINVAL, "max_steps must be >= 1");
    if (run->block < 0 || run->block > 1024 || (run->block % 64) != 0)
        return fail(RDDMC_EINVAL, "block must be a multiple of 64 in [64, 1024] (or 0)");
    if (run->block > 256) return fail(RDDMC_EINVAL, "the walk kernel is built for blocks of at most 256 lanes");
    if (run->grid < 0 || run->chunk < 0) return fail(RDDMC_EINVAL, "negative grid or chunk");
    const uint64_t total = L.h.total_packets;
    if (run->first > total) return fail(RDDMC_EINVAL, "first beyond the batch's packets");
    const uint64_t count = run->count ? run->count : total - run->first;
    if (count > total - run->first) return fail(RDDMC_EINVAL, "first + count beyond the batch's packets");
    if (count == 0) return RDDMC_OK;
    if (L.h.geometry == RDDMC_CART3D) {
        hipError_t e = launch_walk3d(static_cast<const uint8_t *>(d_tables), L.h, *run, run->first, count,
                                     static_cast<unsigned long long *>(d_tally),
                                     static_cast<unsigned long long *>(d_work), reinterpret_cast<hipStream_t>(stream));
        return e == hipSuccess ? RDDMC_OK : hip_fail(e, "3D walk kernel");
    }
    if (L.h.hybrid1d) {
        if (run->surrogate)
            return fail(RDDMC_EUNSUPPORTED, "the escape surrogate runs with pure-DDMC 1D batches only");
        hipError_t e = launch_walk1dh(static_cast<const uint8_t *>(d_tables), L.h, *run, run->first, count,
                                      static_cast<unsigned long long *>(d_tally),
                                      static_cast<unsigned long long *>(d_work), reinterpret_cast<hipStream_t>(stream));
        return e == hipSuccess ? RDDMC_OK : hip_fail(e, "1D hybrid walk kernel");
    }
    hipError_t e = launch_walk(static_cast<const uint8_t *>(d_tables), L.h, L.clouds.data(), *run, run->first,
                               count, static_cast<unsigned long long *>(d_tally),
                               static_cast<unsigned long long *>(d_work), work_bytes,
                               reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? RDDMC_OK : hip_fail(e, "walk kernel");
}

rddmc_status rddmc_tally(const rddmc_batch *batch, const void *d_tally, size_t tally_bytes, rddmc_tally_out *out,
                         void *stream)
{
    Layout L;
    rddmc_status st = make_layout(batch, L);
    if (st != RDDMC_OK) return st;
    if (!d_tally || !out) return fail(RDDMC_EINVAL, "NULL argument");
    if (tally_bytes < L.tally_words * 8) return fail(RDDMC_ESIZE, "tally buffer too small");
    std::vector<uint64_t> h(L.tally_words);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(h.data(), d_tally, L.tally_words * 8, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(tally)");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    for (int ci = 0; ci < L.h.n_clouds; ++ci) {
        const DevCloud &c = L.clouds[ci];
        const uint64_t *w = h.data() + c.tally_off;
        const uint64_t nspec = (uint64_t)c.n_rows * (c.nb + 2);
        if (out->spectrum && out->spectrum[ci]) std::memcpy(out->spectrum[ci], w + kTallyHeader, 8 * nspec);
        if (out->time_hist && out->time_hist[ci])
            std::memcpy(out->time_hist[ci], w + kTallyHeader + nspec, 8 * (RDDMC_TIME_BINS + 2));
        if (out->step_hist && out->step_hist[ci])
            std::memcpy(out->step_hist[ci], w + kTallyHeader + nspec + RDDMC_TIME_BINS + 2, 8 * RDDMC_STEP_BINS);
        if (out->pixels && out->pixels[ci] && c.n_pix)
            std::memcpy(out->pixels[ci], w + kTallyHeader + nspec + RDDMC_TIME_BINS + 2 + RDDMC_STEP_BINS,
                        8 * c.n_pix);
        if (out->stats) {
            rddmc_cloud_stats &z = out->stats[ci];
            z.launched = w[TW_LAUNCHED];
            z.escaped = w[TW_ESCAPED];
            z.capped = w[TW_CAPPED];
            z.steps_total = w[TW_STEPS];
            z.steps_max = w[TW_STEPS_MAX];
            const double done = (double)(z.escaped + z.capped);
            z.steps_mean = done > 0 ? (double)z.steps_total / done : 0.0;
            const double ne = (double)z.escaped;
            const double tsum = (double)w[TW_TSUM] / kTimeFix;
            const long double t2 = ((long double)w[TW_T2_HI] * 18446744073709551616.0L + (long double)w[TW_T2_LO]) /
                                   (long double)kTimeFix;
            z.t_mean = ne > 0 ? tsum / ne : 0.0;
            z.t_var = ne > 0 ? (double)(t2 / (long double)ne) - z.t_mean * z.t_mean : 0.0;
            z.n_rows = c.n_rows;
            z.n_slots = c.nb + 2;
            z.to_mc = w[TW_TO_MC];
            z.to_ddmc = w[TW_TO_DDMC];
            z.reflected = w[TW_REFLECTED];
            z.mc_steps = w[TW_MC_STEPS];
            z.surrogate_calls = w[TW_SURR_CALLS];
            z.absorbed = w[TW_ABSORBED];
            z.n_pix = c.n_pix;
            z.escaped_w = z.t_mean_w = z.t_var_w = 0.0;
            if (c.dust_weight) {
                const uint64_t *ww = w + c.wspec_off;
                long double sw = 0.0L;
                for (uint64_t i = 0; i < nspec; ++i) sw += (long double)ww[4 + i];
                sw /= (long double)kWeightFix;
                const long double two64 = 18446744073709551616.0L;
                const long double swt = ((long double)ww[1] * two64 + (long double)ww[0]) / (long double)kWeightFix;
                const long double swt2 = ((long double)ww[3] * two64 + (long double)ww[2]) / (long double)kTimeFix;
                z.escaped_w = (double)sw;
                if (sw > 0.0L) {
                    z.t_mean_w = (double)(swt / sw);
                    z.t_var_w = (double)(swt2 / sw) - z.t_mean_w * z.t_mean_w;
                }
            }
        }
        if (c.dust_weight && out->spectrum_w && out->spectrum_w[ci])
            std::memcpy(out->spectrum_w[ci], w + c.wspec_off + 4, 8 * nspec);
        if (c.dust_weight && out->spectrum_w2 && out->spectrum_w2[ci])
            std::memcpy(out->spectrum_w2[ci], w + c.wspec_off + 4 + nspec, 8 * nspec);
        if (c.n_census > 0 && out->census_bin && out->census_bin[ci])
            std::memcpy(out->census_bin[ci], w + c.census_bin_off, 8ull * (c.n_census + 1) * c.n_states);
        if (c.n_census > 0 && out->census_path && out->census_path[ci])
            std::memcpy(out->census_path[ci], w + c.census_path_off, 8ull * c.n_census * c.n_states);
        if (c.n_census > 0 && out->census_accel && out->census_accel[ci])
            std::memcpy(out->census_accel[ci], w + c.census_accel_off, 8ull * c.n_census * c.nc);
    }
    return RDDMC_OK;
}

rddmc_status rddmc_read_tables(const rddmc_batch *batch, const void *d_tables, int32_t cloud, double *k,
                               double *rates, void *hot, void *lo_words, void *stream)
{
    Layout L;
    rddmc_status st = make_layout(batch, L);
    if (st != RDDMC_OK) return st;
    if (!d_tables) return fail(RDDMC_EINVAL, "d_tables is NULL");
    if (cloud < 0 || cloud >= L.h.n_clouds) return fail(RDDMC_EINVAL, "cloud index out of range");
    const DevCloud &c = L.clouds[cloud];
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uint8_t *base = static_cast<const uint8_t *>(d_tables);
    hipError_t e;
    if (k && (e = hipMemcpyAsync(k, base + c.off_k, 8 * c.n_states, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "read k");
    if (rates) {
        if (!c.keep_rates) return fail(RDDMC_EINVAL, "rates were not kept (RDDMC_FLAG_KEEP_RATES)");
        if ((e = hipMemcpyAsync(rates, base + c.off_rates, 8 * c.n_states * (c.nf + 2), hipMemcpyDeviceToHost, s)) !=
            hipSuccess)
            return hip_fail(e, "read rates");
    }
    if (hot && (e = hipMemcpyAsync(hot, base + c.off_hot, sizeof(HotRecord) * c.n_states, hipMemcpyDeviceToHost,
                                   s)) != hipSuccess)
        return hip_fail(e, "read hot");
    if (lo_words && (e = hipMemcpyAsync(lo_words, base + c.off_lo_words, 16 * c.n_states, hipMemcpyDeviceToHost,
                                        s)) != hipSuccess)
        return hip_fail(e, "read lo words");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return RDDMC_OK;
}

rddmc_status rddmc_read_redistribution(const rddmc_batch *batch, const void *d_tables, int32_t cloud, double *prob,
                                       uint32_t *alias, void *stream)
{
    Layout L;
    rddmc_status st = make_layout(batch, L);
    if (st != RDDMC_OK) return st;
    if (!d_tables) return fail(RDDMC_EINVAL, "d_tables is NULL");
    if (cloud < 0 || cloud >= L.h.n_clouds) return fail(RDDMC_EINVAL, "cloud index out of range");
    const DevCloud &c = L.clouds[cloud];
    if (!c.groups) return fail(RDDMC_EINVAL, "cloud %d has no frequency groups (RDDMC_FLAG_GROUPS)", cloud);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uint8_t *base = static_cast<const uint8_t *>(d_tables);
    const uint64_t n = (uint64_t)c.nb * c.nb;
    hipError_t e;
    if (prob && (e = hipMemcpyAsync(prob, base + c.off_grp_prob, 8 * n, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "read redistribution probabilities");
    if (alias && (e = hipMemcpyAsync(alias, base + c.off_grp_alias, 8 * n, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "read alias tables");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return RDDMC_OK;
}

/* ---- learned escape surrogate: data, windows, per-state tables ------------------------- */

namespace {

// The surrogate window of one 1D cloud: interior cells of a uniform (k0, T) cloud whose
// optical width, face geometry and Doppler shifts lie in the trained domain (the longest
// contiguous run), times the contiguous bins around x = 0 with centres within x_core and
// widths in the domain.  Empty (i_hi < i_lo) when nothing qualifies.
SurrCloud surrogate_window(const rddmc_medium &m, const rddmc_surrogate_cfg &cfg)
{
    SurrCloud w{0, -1, 0, -1, 0, 0};
    if (m.geometry != RDDMC_SLAB && m.geometry != RDDMC_SPHERE) return w;
    const int nc = m.n_cells[0], nb = m.n_bins;
    if (nc < 3) return w;
    for (int i = 1; i < nc; ++i)
        if (m.k0[i] != m.k0[0] || m.temp[i] != m.temp[0]) return w;
    const double T = m.temp[0];
    const double a = 4.702e-4 * std::sqrt(1.0e4 / T), vth = 12.85 * std::sqrt(T / 1.0e4);
    if (!(a >= cfg.a_min && a <= cfg.a_max)) return w;
    const double *f = m.faces[0];
    int best_lo = 0, best_len = 0, run_lo = 0, run_len = 0;
    for (int i = 1; i <= nc - 2; ++i) {
        const double lo = f[i], hi = f[i + 1], wd = hi - lo;
        const double tau = m.k0[i] * wd;
        double g0 = 1.0, g1 = 1.0;
        if (m.geometry == RDDMC_SPHERE) {
            const double v3 = (hi * hi * hi - lo * lo * lo) / 3.0;
            g0 = lo * lo / v3 * wd;
            g1 = hi * hi / v3 * wd;
        }
        double s0 = 0.0, s1 = 0.0;
        if (m.vel) {
            s0 = -m.f_mu * (m.vel[i] - m.vel[i - 1]) / vth;
            s1 = -m.f_mu * (m.vel[i + 1] - m.vel[i]) / vth;
        }
        const bool ok = tau >= cfg.tau_min && tau <= cfg.tau_max && g0 >= cfg.g_min && g0 <= cfg.g_max &&
                        g1 >= cfg.g_min && g1 <= cfg.g_max && std::fabs(s0) <= cfg.shift_max &&
                        std::fabs(s1) <= cfg.shift_max;
        if (ok) {
            if (run_len == 0) run_lo = i;
            ++run_len;
            if (run_len > best_len) {
                best_len = run_len;
                best_lo = run_lo;
            }
        } else {
            run_len = 0;
        }
    }
    if (best_len == 0) return w;
    const double *e = m.bin_edges;
    int j0 = 0;      // bin whose centre is nearest x = 0
    for (int j = 1; j < nb; ++j)
        if (std::fabs(0.5 * (e[j] + e[j + 1])) < std::fabs(0.5 * (e[j0] + e[j0 + 1]))) j0 = j;
    auto bin_ok = [&](int j) {
        const double c = 0.5 * (e[j] + e[j + 1]), dx = e[j + 1] - e[j];
        return std::fabs(c) <= cfg.x_core && dx >= cfg.dx_min && dx <= cfg.dx_max;
    };
    if (!bin_ok(j0)) return w;
    int jl = j0, jh = j0;
    while (jl > 0 && bin_ok(jl - 1)) --jl;
    while (jh < nb - 1 && bin_ok(jh + 1)) ++jh;
    w.i_lo = best_lo;
    w.i_hi = best_lo + best_len - 1;
    w.j_lo = jl;
    w.j_hi = jh;
    return w;
}

struct SurrLayout {
    SurrHeader h{};
    std::vector<SurrCloud> clouds;
    uint64_t off_x = 0, off_sw = 0, bytes = 0;
};

rddmc_status surrogate_layout(const rddmc_batch *b, const rddmc_surrogate_cfg *cfg, int64_t max_batch,
                              SurrLayout &S)
{
    if (!cfg) return fail(RDDMC_EINVAL, "cfg is NULL");
    if (max_batch < 1 || max_batch > (1ll << 24)) return fail(RDDMC_EINVAL, "max_batch must be in [1, 2^24]");
    Layout L;
    rddmc_status st = make_layout(b, L);
    if (st != RDDMC_OK) return st;
    if (L.h.hybrid1d) return fail(RDDMC_EUNSUPPORTED, "the escape surrogate runs with pure-DDMC 1D batches only");
    const int n = b->n_clouds;
    S.clouds.resize(n);
    uint64_t rec = 0;
    for (int c = 0; c < n; ++c) {
        SurrCloud w = surrogate_window(b->clouds[c], *cfg);
        w.rec_off = rec;
        if (w.i_hi >= w.i_lo) rec += (uint64_t)(w.i_hi - w.i_lo + 1) * (w.j_hi - w.j_lo + 1);
        S.clouds[c] = w;
    }
    const int64_t cap = (max_batch + 31) & ~31ll;
    uint64_t off = align_up(sizeof(SurrHeader));
    S.h.n_clouds = n;
    S.h.off_clouds = off;
    off = align_up(off + sizeof(SurrCloud) * n);
    S.off_x = off;
    off = align_up(off + 4ull * kSurrIn * cap);
    S.off_sw = off;
    off = align_up(off + 8ull * cap);
    S.h.off_records = off;
    S.h.n_records = rec;
    S.bytes = off + 4ull * kSurrRec * rec;
    return RDDMC_OK;
}

}  // namespace

rddmc_status rddmc_surrogate_bytes(const rddmc_batch *batch, const rddmc_surrogate_cfg *cfg, int64_t max_batch,
                                   size_t *bytes, uint64_t *n_states)
{
    if (!bytes) return fail(RDDMC_EINVAL, "bytes is NULL");
    SurrLayout S;
    rddmc_status st = surrogate_layout(batch, cfg, max_batch, S);
    if (st != RDDMC_OK) return st;
    *bytes = S.bytes;
    if (n_states) *n_states = S.h.n_records;
    return RDDMC_OK;
}

rddmc_status rddmc_surrogate_window(const rddmc_batch *batch, const rddmc_surrogate_cfg *cfg, int32_t cloud,
                                    int32_t *window)
{
    if (!batch || !window || cloud < 0 || cloud >= batch->n_clouds) return fail(RDDMC_EINVAL, "bad arguments");
    if (!cfg) return fail(RDDMC_EINVAL, "cfg is NULL");
    const SurrCloud w = surrogate_window(batch->clouds[cloud], *cfg);
    window[0] = w.i_lo;
    window[1] = w.i_hi;
    window[2] = w.j_lo;
    window[3] = w.j_hi;
    return RDDMC_OK;
}

rddmc_status rddmc_surrogate_attach(const rddmc_batch *batch, const void *d_tables, void *d_params, void *d_work,
                                    int64_t max_batch, const rddmc_surrogate_cfg *cfg, void *d_surr, size_t bytes,
                                    void *stream)
{
    SurrLayout S;
    rddmc_status st = surrogate_layout(batch, cfg, max_batch, S);
    if (st != RDDMC_OK) return st;
    if (!d_tables || !d_params || !d_work || !d_surr) return fail(RDDMC_EINVAL, "NULL argument");
    if ((uintptr_t)d_surr % kAlign) return fail(RDDMC_EINVAL, "d_surr must be 256-byte aligned");
    if (bytes < S.bytes) return fail(RDDMC_ESIZE, "surrogate buffer %zu < required %llu", bytes,
                                     (unsigned long long)S.bytes);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::vector<uint8_t> hdr(S.off_x, 0);
    std::memcpy(hdr.data(), &S.h, sizeof S.h);
    std::memcpy(hdr.data() + S.h.off_clouds, S.clouds.data(), sizeof(SurrCloud) * S.clouds.size());
    uint8_t *base = static_cast<uint8_t *>(d_surr);
    hipError_t e = hipMemcpyAsync(base, hdr.data(), hdr.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(surrogate header)");
    const int64_t cap = (max_batch + 31) & ~31ll;
    float *X = reinterpret_cast<float *>(base + S.off_x);
    float *SW = reinterpret_cast<float *>(base + S.off_sw);
    float *R = reinterpret_cast<float *>(base + S.h.off_records);
    for (uint64_t first = 0; first < S.h.n_records; first += (uint64_t)max_batch) {
        const uint64_t cnt = std::min<uint64_t>((uint64_t)max_batch, S.h.n_records - first);
        if ((e = launch_surr_features(static_cast<const uint8_t *>(d_tables), base, first, cnt, X, SW, s)) !=
            hipSuccess)
            return hip_fail(e, "surrogate features");
        if ((e = mdn_forward(d_params, d_work, cap, X, (int)cnt, nullptr, s)) != hipSuccess)
            return hip_fail(e, "surrogate inference");
        if ((e = launch_surr_records(mdn_outputs(d_work, cap), SW, cnt, R + first * kSurrRec, s)) != hipSuccess)
            return hip_fail(e, "surrogate records");
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return RDDMC_OK;
}

rddmc_status rddmc_surrogate_samples(const rddmc_batch *batch, const void *d_tables, const int32_t *h_cloud,
                                     const int32_t *h_state, int64_t n, uint64_t seed, uint64_t max_steps,
                                     void *d_scratch, size_t scratch_bytes, float *d_x, float *d_y,
                                     uint64_t *d_steps, void *stream)
{
    Layout L;
    rddmc_status st = make_layout(batch, L);
    if (st != RDDMC_OK) return st;
    if (!d_tables || !h_cloud || !h_state || !d_scratch || !d_x || !d_y || !d_steps)
        return fail(RDDMC_EINVAL, "NULL argument");
    if (n < 1) return fail(RDDMC_EINVAL, "n < 1");
    if (scratch_bytes < 8ull * (uint64_t)n) return fail(RDDMC_ESIZE, "scratch needs 8 n bytes");
    if (max_steps < 1) return fail(RDDMC_EINVAL, "max_steps must be >= 1");
    if (L.h.geometry == RDDMC_CART3D || L.h.hybrid1d)
        return fail(RDDMC_EUNSUPPORTED, "sub-walk data is built for pure-DDMC 1D clouds");
    bool moving = false;
    for (int64_t q = 0; q < n; ++q) {
        const int c = h_cloud[q];
        if (c < 0 || c >= batch->n_clouds) return fail(RDDMC_EINVAL, "sample %lld: bad cloud", (long long)q);
        const DevCloud &dc = L.clouds[c];
        const int i = h_state[q] / dc.nb;
        if (h_state[q] < 0 || (uint64_t)h_state[q] >= dc.n_states || i < 1 || i > dc.nc - 2)
            return fail(RDDMC_EINVAL, "sample %lld: the start state must lie in a cell with two neighbours",
                        (long long)q);
        moving |= dc.moving != 0;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int32_t *dc = static_cast<int32_t *>(d_scratch);
    int32_t *ds = dc + n;
    hipError_t e = hipMemcpyAsync(dc, h_cloud, 4ull * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ds, h_state, 4ull * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_subwalk(static_cast<const uint8_t *>(d_tables), moving, seed, max_steps, dc, ds, n, d_x, d_y,
                           reinterpret_cast<unsigned long long *>(d_steps), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // the host start arrays are read asynchronously
    return e == hipSuccess ? RDDMC_OK : hip_fail(e, "sub-walk kernel");
}

/* ---- exact per-cell exit kernel -------------------------------------------------------- */

namespace {

constexpr uint64_t kEkChunk = 16384;  // window states per row-kernel launch
constexpr int kEkArraysHost = 7;      // per-bin chain arrays per cell (exitkernel.hip)

struct EkPlan {
    SurrHeader h{};
    std::vector<SurrCloud> clouds;
    std::vector<ExitRec> recs;
    uint64_t bytes = 0;
};

struct EkScratch {
    uint64_t cb = 0, mn = 0, sc = 0, sp = 0, total = 0;   // offsets and size
};

void ek_scratch_layout(const Layout &L, EkScratch &S)
{
    uint64_t need_cb = 0, need_nb = 0;
    for (const DevCloud &c : L.clouds) {
        need_cb = std::max<uint64_t>(need_cb, 8ull * kEkArraysHost * c.nc * c.nb);
        need_nb = std::max<uint64_t>(need_nb, (uint64_t)c.nb);
    }
    S.cb = 0;
    S.mn = align_up(need_cb);
    S.sc = align_up(S.mn + 8ull * need_nb);
    S.sp = align_up(S.sc + 24ull * need_nb * kEkChunk);
    S.total = align_up(S.sp + 8ull * kEkChunk);
}

rddmc_status ek_check(const rddmc_batch *b, const rddmc_exitkernel_cfg *cfg, Layout &L)
{
    if (!cfg) return fail(RDDMC_EINVAL, "cfg is NULL");
    if (!(cfg->min_steps >= 1.0) || !std::isfinite(cfg->min_steps))
        return fail(RDDMC_EINVAL, "min_steps must be finite and >= 1");
    if (!(cfg->tail >= 0.0 && cfg->tail <= 1e-6)) return fail(RDDMC_EINVAL, "tail must lie in [0, 1e-6]");
    rddmc_status st = make_layout(b, L);
    if (st != RDDMC_OK) return st;
    if (L.h.geometry == RDDMC_CART3D || L.h.hybrid1d)
        return fail(RDDMC_EUNSUPPORTED, "the exit kernel runs with pure-DDMC 1D batches only");
    return RDDMC_OK;
}

// Windows (interior cells x the contiguous bins around the longest expected sub-walk where every
// window cell's expected sub-walk is at least min_steps) and each window state's kept exit-bin
// span.  Runs kernels and synchronises.
rddmc_status ek_plan(const rddmc_batch *b, const Layout &L, const void *d_tables, const rddmc_exitkernel_cfg &cfg,
                     uint8_t *scr, const EkScratch &X, hipStream_t s, EkPlan &P)
{
    const int n = b->n_clouds;
    P.clouds.assign(n, SurrCloud{0, -1, 0, -1, 0, 0});
    P.recs.clear();
    uint64_t row = 0;
    double *cb = reinterpret_cast<double *>(scr + X.cb);
    double *mn = reinterpret_cast<double *>(scr + X.mn);
    double *sc = reinterpret_cast<double *>(scr + X.sc);
    int2 *sp = reinterpret_cast<int2 *>(scr + X.sp);
    const uint8_t *tb = static_cast<const uint8_t *>(d_tables);
    hipError_t e;
    for (int ci = 0; ci < n; ++ci) {
        const DevCloud &c = L.clouds[ci];
        SurrCloud w{0, -1, 0, -1, (uint64_t)P.recs.size(), 0};
        // a sphere's innermost cell is interior when its inner face is the centre (no leak
        // through it); any other first cell borders the inner boundary
        const bool centre = c.geometry == RDDMC_SPHERE && b->clouds[ci].faces[0][0] == 0.0;
        const int i_lo = centre ? 0 : 1, i_hi = c.nc - 2;
        if (i_hi >= i_lo) {
            if ((e = launch_ek_prep(tb, c, cb, s)) != hipSuccess) return hip_fail(e, "exit kernel: chain arrays");
            if ((e = launch_ek_minsteps(cb, c.nc, c.nb, i_lo, i_hi, mn, s)) != hipSuccess)
                return hip_fail(e, "exit kernel: sub-walk lengths");
            std::vector<double> h(c.nb);
            if ((e = hipMemcpyAsync(h.data(), mn, 8ull * c.nb, hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return hip_fail(e, "exit kernel: sub-walk lengths read-back");
            int j0 = 0;
            for (int j = 1; j < c.nb; ++j)
                if (h[j] > h[j0]) j0 = j;
            if (h[j0] >= cfg.min_steps) {
                int jl = j0, jh = j0;
                while (jl > 0 && h[jl - 1] >= cfg.min_steps) --jl;
                while (jh < c.nb - 1 && h[jh + 1] >= cfg.min_steps) ++jh;
                w.i_lo = i_lo;
                w.i_hi = i_hi;
                w.j_lo = jl;
                w.j_hi = jh;
                const int nj = jh - jl + 1;
                const uint64_t nst = (uint64_t)(i_hi - i_lo + 1) * nj;
                std::vector<int2> span(kEkChunk);
                for (uint64_t q0 = 0; q0 < nst; q0 += kEkChunk) {
                    const uint64_t cnt = std::min<uint64_t>(kEkChunk, nst - q0);
                    if ((e = launch_ek_rows(cb, c.nc, c.nb, i_lo, jl, nj, q0, cnt, cfg.tail, sc, sp, nullptr, nullptr,
                                            s)) != hipSuccess)
                        return hip_fail(e, "exit kernel: row spans");
                    if ((e = hipMemcpyAsync(span.data(), sp, 8ull * cnt, hipMemcpyDeviceToHost, s)) != hipSuccess ||
                        (e = hipStreamSynchronize(s)) != hipSuccess)
                        return hip_fail(e, "exit kernel: row spans read-back");
                    for (uint64_t t = 0; t < cnt; ++t) {
                        const int m = span[t].y;
                        if (m < 1 || span[t].x < 0 || span[t].x + m > c.nb)
                            return fail(RDDMC_ENUMERIC, "exit kernel: cloud %d has an empty exit law", ci);
                        P.recs.push_back(ExitRec{row, span[t].x, m});
                        row += 24ull * m;
                    }
                }
            }
        }
        P.clouds[ci] = w;
    }
    P.h.n_clouds = n;
    P.h.kind = kSurrExact;
    P.h.off_clouds = align_up(sizeof(SurrHeader));
    P.h.off_records = align_up(P.h.off_clouds + sizeof(SurrCloud) * n);
    P.h.n_records = P.recs.size();
    P.h.off_rows = align_up(P.h.off_records + sizeof(ExitRec) * P.recs.size());
    P.bytes = P.h.off_rows + row;
    return RDDMC_OK;
}

}  // namespace

rddmc_status rddmc_exitkernel_scratch_bytes(const rddmc_batch *batch, size_t *bytes)
{
    if (!bytes) return fail(RDDMC_EINVAL, "bytes is NULL");
    Layout L;
    rddmc_status st = make_layout(batch, L);
    if (st != RDDMC_OK) return st;
    EkScratch X;
    ek_scratch_layout(L, X);
    *bytes = X.total;
    return RDDMC_OK;
}

rddmc_status rddmc_exitkernel_bytes(const rddmc_batch *batch, const void *d_tables, const rddmc_exitkernel_cfg *cfg,
                                    void *d_scratch, size_t scratch_bytes, size_t *bytes, uint64_t *n_states,
                                    int32_t *h_windows, void *stream)
{
    Layout L;
    rddmc_status st = ek_check(batch, cfg, L);
    if (st != RDDMC_OK) return st;
    if (!d_tables || !d_scratch || !bytes) return fail(RDDMC_EINVAL, "NULL argument");
    EkScratch X;
    ek_scratch_layout(L, X);
    if ((uintptr_t)d_scratch % kAlign) return fail(RDDMC_EINVAL, "d_scratch must be 256-byte aligned");
    if (scratch_bytes < X.total)
        return fail(RDDMC_ESIZE, "scratch %zu < required %llu", scratch_bytes, (unsigned long long)X.total);
    EkPlan P;
    st = ek_plan(batch, L, d_tables, *cfg, static_cast<uint8_t *>(d_scratch), X, reinterpret_cast<hipStream_t>(stream),
                 P);
    if (st != RDDMC_OK) return st;
    *bytes = P.bytes;
    if (n_states) *n_states = P.h.n_records;
    if (h_windows)
        for (int c = 0; c < batch->n_clouds; ++c) {
            h_windows[4 * c + 0] = P.clouds[c].i_lo;
            h_windows[4 * c + 1] = P.clouds[c].i_hi;
            h_windows[4 * c + 2] = P.clouds[c].j_lo;
            h_windows[4 * c + 3] = P.clouds[c].j_hi;
        }
    return RDDMC_OK;
}

rddmc_status rddmc_exitkernel_build(const rddmc_batch *batch, const void *d_tables, const rddmc_exitkernel_cfg *cfg,
                                    void *d_scratch, size_t scratch_bytes, void *d_ek, size_t bytes, void *stream)
{
    Layout L;
    rddmc_status st = ek_check(batch, cfg, L);
    if (st != RDDMC_OK) return st;
    if (!d_tables || !d_scratch || !d_ek) return fail(RDDMC_EINVAL, "NULL argument");
    if ((uintptr_t)d_scratch % kAlign || (uintptr_t)d_ek % kAlign)
        return fail(RDDMC_EINVAL, "d_scratch and d_ek must be 256-byte aligned");
    EkScratch X;
    ek_scratch_layout(L, X);
    if (scratch_bytes < X.total)
        return fail(RDDMC_ESIZE, "scratch %zu < required %llu", scratch_bytes, (unsigned long long)X.total);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint8_t *scr = static_cast<uint8_t *>(d_scratch);
    EkPlan P;
    st = ek_plan(batch, L, d_tables, *cfg, scr, X, s, P);
    if (st != RDDMC_OK) return st;
    if (bytes < P.bytes)
        return fail(RDDMC_ESIZE, "exit-kernel buffer %zu < required %llu", bytes, (unsigned long long)P.bytes);
    uint8_t *base = static_cast<uint8_t *>(d_ek);
    std::vector<uint8_t> hdr(P.h.off_rows, 0);
    std::memcpy(hdr.data(), &P.h, sizeof P.h);
    std::memcpy(hdr.data() + P.h.off_clouds, P.clouds.data(), sizeof(SurrCloud) * P.clouds.size());
    if (!P.recs.empty()) std::memcpy(hdr.data() + P.h.off_records, P.recs.data(), sizeof(ExitRec) * P.recs.size());
    hipError_t e = hipMemcpyAsync(base, hdr.data(), hdr.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(exit-kernel header)");
    double *cb = reinterpret_cast<double *>(scr + X.cb);
    double *sc = reinterpret_cast<double *>(scr + X.sc);
    const uint8_t *tb = static_cast<const uint8_t *>(d_tables);
    const ExitRec *recs = reinterpret_cast<const ExitRec *>(base + P.h.off_records);
    for (int ci = 0; ci < batch->n_clouds; ++ci) {
        const SurrCloud &w = P.clouds[ci];
        if (w.i_hi < w.i_lo) continue;
        const DevCloud &c = L.clouds[ci];
        if ((e = launch_ek_prep(tb, c, cb, s)) != hipSuccess) return hip_fail(e, "exit kernel: chain arrays");
        const int nj = w.j_hi - w.j_lo + 1;
        const uint64_t nst = (uint64_t)(w.i_hi - w.i_lo + 1) * nj;
        for (uint64_t q0 = 0; q0 < nst; q0 += kEkChunk) {
            const uint64_t cnt = std::min<uint64_t>(kEkChunk, nst - q0);
            if ((e = launch_ek_rows(cb, c.nc, c.nb, w.i_lo, w.j_lo, nj, q0, cnt, cfg->tail, sc, nullptr,
                                    recs + w.rec_off, base + P.h.off_rows, s)) != hipSuccess)
                return hip_fail(e, "exit kernel: rows");
        }
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return RDDMC_OK;
}

rddmc_status rddmc_exitlaw_samples(const rddmc_batch *batch, const void *d_tables, const int32_t *h_cloud,
                                   const int32_t *h_state, const int32_t *h_count, int64_t n_pairs, uint64_t seed,
                                   void *d_scratch, size_t scratch_bytes, float *d_x, float *d_y, void *stream)
{
    Layout L;
    rddmc_status st = make_layout(batch, L);
    if (st != RDDMC_OK) return st;
    if (!d_tables || !h_cloud || !h_state || !h_count || !d_scratch || !d_x || !d_y)
        return fail(RDDMC_EINVAL, "NULL argument");
    if (n_pairs < 1) return fail(RDDMC_EINVAL, "n_pairs < 1");
    if (L.h.geometry == RDDMC_CART3D || L.h.hybrid1d)
        return fail(RDDMC_EUNSUPPORTED, "exact exit-law samples are drawn for pure-DDMC 1D clouds");
    int nb_max = 0;
    std::vector<int64_t> off(n_pairs);
    int64_t rows = 0;
    for (int64_t q = 0; q < n_pairs; ++q) {
        const int c = h_cloud[q];
        if (c < 0 || c >= batch->n_clouds) return fail(RDDMC_EINVAL, "pair %lld: bad cloud", (long long)q);
        const DevCloud &dc = L.clouds[c];
        const int i = h_state[q] / dc.nb;
        if (h_state[q] < 0 || (uint64_t)h_state[q] >= dc.n_states || i < 1 || i > dc.nc - 2)
            return fail(RDDMC_EINVAL, "pair %lld: the state must lie in a cell with two neighbours", (long long)q);
        if (h_count[q] < 0) return fail(RDDMC_EINVAL, "pair %lld: negative count", (long long)q);
        nb_max = std::max(nb_max, dc.nb);
        off[q] = rows;
        rows += h_count[q];
    }
    const uint64_t n = (uint64_t)n_pairs;
    const uint64_t o_pc = 0, o_ps = align_up(4 * n), o_cnt = align_up(o_ps + 4 * n), o_off = align_up(o_cnt + 4 * n),
                   o_scr = align_up(o_off + 8 * n), need = o_scr + 88ull * nb_max * n;
    if (scratch_bytes < need)
        return fail(RDDMC_ESIZE, "scratch %zu < required %llu", scratch_bytes, (unsigned long long)need);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint8_t *scr = static_cast<uint8_t *>(d_scratch);
    hipError_t e = hipMemcpyAsync(scr + o_pc, h_cloud, 4 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(scr + o_ps, h_state, 4 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(scr + o_cnt, h_count, 4 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(scr + o_off, off.data(), 8 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_ek_samples(static_cast<const uint8_t *>(d_tables), reinterpret_cast<const int32_t *>(scr + o_pc),
                              reinterpret_cast<const int32_t *>(scr + o_ps), reinterpret_cast<const int32_t *>(scr + o_cnt),
                              reinterpret_cast<const int64_t *>(scr + o_off), n, seed, nb_max,
                              reinterpret_cast<double *>(scr + o_scr), d_x, d_y, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // the host arrays are read asynchronously
    return e == hipSuccess ? RDDMC_OK : hip_fail(e, "exit-law samples");
}

/* ---- mixture-density network of the escape surrogate --------------------------------- */

rddmc_status rddmc_mdn_bytes(int64_t max_batch, size_t *param_bytes, size_t *work_bytes, int64_t *n_params)
{
    if (max_batch < 1 || max_batch > (1ll << 24)) return fail(RDDMC_EINVAL, "max_batch must be in [1, 2^24]");
    const int64_t cap = (max_batch + 31) & ~31ll;
    if (param_bytes) *param_bytes = mdn_param_bytes();
    if (work_bytes) *work_bytes = mdn_work_bytes(cap);
    if (n_params) *n_params = mdn_n_params();
    return RDDMC_OK;
}

rddmc_status rddmc_mdn_init(void *d_params, uint64_t seed, void *stream)
{
    if (!d_params) return fail(RDDMC_EINVAL, "d_params is NULL");
    hipError_t e = mdn_init(d_params, seed, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? RDDMC_OK : hip_fail(e, "mdn init");
}

rddmc_status rddmc_mdn_set(void *d_params, const float *h_theta, void *stream)
{
    if (!d_params || !h_theta) return fail(RDDMC_EINVAL, "NULL argument");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = mdn_n_params();
    hipError_t e = mdn_init(d_params, 0, s);        // zero the optimiser state
    if (e == hipSuccess) e = hipMemcpyAsync(d_params, h_theta, 4ull * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = mdn_refresh(d_params, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? RDDMC_OK : hip_fail(e, "mdn set");
}

rddmc_status rddmc_mdn_get(const void *d_params, float *h_theta, float *h_grad, void *stream)
{
    if (!d_params) return fail(RDDMC_EINVAL, "d_params is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = mdn_n_params();
    const float *f = static_cast<const float *>(d_params);
    hipError_t e = hipSuccess;
    if (h_theta) e = hipMemcpyAsync(h_theta, f, 4ull * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && h_grad) e = hipMemcpyAsync(h_grad, f + 3 * n, 4ull * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? RDDMC_OK : hip_fail(e, "mdn get");
}

rddmc_status rddmc_mdn_forward(void *d_params, void *d_work, int64_t max_batch, const float *d_x, int32_t n,
                               float *d_out, void *stream)
{
    if (!d_params || !d_work || !d_x) return fail(RDDMC_EINVAL, "NULL argument");
    if (n < 1 || n > max_batch) return fail(RDDMC_EINVAL, "n must be in [1, max_batch]");
    const int64_t cap = (max_batch + 31) & ~31ll;
    hipError_t e = mdn_forward(d_params, d_work, cap, d_x, n, d_out, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? RDDMC_OK : hip_fail(e, "mdn forward");
}

rddmc_status rddmc_mdn_loss_grad(void *d_params, void *d_work, int64_t max_batch, const float *d_x,
                                 const float *d_y, int32_t n, float *d_loss, void *stream)
{
    if (!d_params || !d_work || !d_x || !d_y) return fail(RDDMC_EINVAL, "NULL argument");
    if (n < 1 || n > max_batch) return fail(RDDMC_EINVAL, "n must be in [1, max_batch]");
    const int64_t cap = (max_batch + 31) & ~31ll;
    hipError_t e = mdn_loss_grad(d_params, d_work, cap, d_x, d_y, n, d_loss, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? RDDMC_OK : hip_fail(e, "mdn loss/grad");
}

rddmc_status rddmc_mdn_adam(void *d_params, int64_t step, float lr, void *stream)
{
    if (!d_params) return fail(RDDMC_EINVAL, "d_params is NULL");
    if (step < 1 || !(lr > 0.0f)) return fail(RDDMC_EINVAL, "step >= 1 and lr > 0 required");
    hipError_t e = mdn_adam(d_params, step, lr, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? RDDMC_OK : hip_fail(e, "mdn adam");
}

rddmc_status rddmc_philox_fill(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                               uint64_t n, uint32_t *d_out, void *stream)
{
    if (!d_out && n) return fail(RDDMC_EINVAL, "d_out is NULL");
    hipError_t e = launch_philox_fill(k0, k1, c0, c1, c2, c3, n, d_out, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? RDDMC_OK : hip_fail(e, "philox kernel");
}

rddmc_status rddmc_transport_static(const rddmc_batch *batch, const void *d_tables, const rddmc_run *run,
                                    void *d_tally, size_t tally_bytes, void *stream)
{
    if (!run) return fail(RDDMC_EINVAL, "NULL argument");
    if (run->grid > 0 && run->block >= 0) {
        const uint64_t block = run->block > 0 ? (uint64_t)run->block : 256;
        const uint64_t lanes = (uint64_t)run->grid * block;
        if (lanes > RDDMC_STATIC_WORK_LANES)
            return fail(RDDMC_ESIZE,
                        "grid x block = %llu resident lanes; the static work area holds export slots for at most "
                        "%llu (RDDMC_STATIC_WORK_LANES)",
                        (unsigned long long)lanes, (unsigned long long)RDDMC_STATIC_WORK_LANES);
    }
    void *work = nullptr;
    rddmc_status st = static_work_of_current_device(&work);
    if (st != RDDMC_OK) return st;
    return rddmc_transport(batch, d_tables, run, d_tally, tally_bytes, work, RDDMC_STATIC_WORK_BYTES, stream);
}

}  // extern "C"
