// checkpoint.hip -- save a sim at an iteration boundary and build a sim from
// such a checkpoint (we_save, we_checkpoint_inspect, we_load).
//
// The WE procedure saves every trajectory's coordinates and weight after each
// iteration (Sec. II.B); an iteration boundary is also a consistent cut of the
// whole computation.  Random numbers are keyed by (seed, slot, event,
// iteration), so a checkpoint needs no generator state: the walkers, the
// device iteration counter, the series and the configuration determine every
// later iteration.
//
// File layout (host byte order):
//   Header (64 bytes): magic "WESIMCKP", version, header size, sizes of the
//     sim, the iteration, the current buffer, a fingerprint of the network,
//     the workspace size;
//   then tagged sections, each (uint32 tag, uint32 0, uint64 bytes, bytes):
//     PARM  scalar parameters (ParamsRec)
//     GRID  coef[S], edges[n_bins+1], coef2[S], edges2[n_bins2+1] (axis 2 only)
//     ARRS  tgt_coef[S], seeds[n_runs], x0[S], x_rec[S], joint[n_joint]
//     WORK  the device workspace, byte for byte (walker buffers, series,
//           histogram accumulators, reweighting flux matrix, counters)
//     NWLK  walkers per run as the host last saw them
//     CMTR  committor: flags, sizes, params, Adam moments, features, edges,
//           transposed weights (empty when untrained)
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "we_internal.h"

namespace {

const char kMagic[8] = {'W', 'E', 'S', 'I', 'M', 'C', 'K', 'P'};
const uint32_t kVersion = 1;

struct Header {
    char magic[8];
    uint32_t version;
    uint32_t header_bytes;
    int32_t S, R, n_runs, NB, M, max_iters, iter, cur;
    uint64_t net_fp;
    uint64_t ws_bytes;
};
static_assert(sizeof(Header) == 64, "checkpoint header is 64 bytes");

struct ParamsRec {
    double tau, tgt_thr, leap_eps;
    int32_t m_targ, n_runs, max_iters, kernel, recycle;
    int32_t hist_species, hist_lo, hist_hi, n_joint, joint_bins, joint_width;
    int32_t record_iters, rw_period, rw_reset, engine, resample_rule;
    int32_t n_bins, n_bins2, hist_iters, walkers_per_wave;   // 0: not the group kernel
};

enum : uint32_t {
    T_PARM = 0x4d524150u, T_GRID = 0x44495247u, T_ARRS = 0x53525241u,
    T_WORK = 0x4b524f57u, T_NWLK = 0x4b4c574eu, T_CMTR = 0x52544d43u
};

// FNV-1a over the network as compiled: sizes, every descriptor field, the
// change lists and the Hill factors.
struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void bytes(const void *p, size_t n) {
        const unsigned char *c = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
    }
    template <class T> void val(T v) { bytes(&v, sizeof v); }
};

uint64_t network_fingerprint(const we_network *net) {
    Fnv f;
    f.val(net->S);
    f.val(net->R);
    for (const RxnDesc &d : net->desc) {
        f.val(d.c); f.val(d.s1); f.val(d.s2); f.val(d.nu1); f.val(d.nu2);
    }
    for (int32_t v : net->chg_ptr) f.val(v);
    for (int32_t v : net->chg) f.val(v);
    for (const HillDesc &hd : net->hill) { f.val(hd.K); f.val(hd.species); f.val(hd.n); }
    return f.h;
}

struct Writer {
    std::vector<char> buf;
    void raw(const void *p, size_t n) { buf.insert(buf.end(), (const char *)p, (const char *)p + n); }
    void section(uint32_t tag, const void *p, size_t n) {
        const uint32_t z = 0;
        const uint64_t nb = n;
        raw(&tag, 4); raw(&z, 4); raw(&nb, 8);
        if (n) raw(p, n);
    }
    template <class T> void section_vec(uint32_t tag, const std::vector<T> &v) {
        section(tag, v.data(), v.size() * sizeof(T));
    }
};

struct Reader {
    std::vector<char> buf;
    size_t pos = 0;
    bool take(void *p, size_t n) {
        if (pos + n > buf.size()) return false;
        std::memcpy(p, buf.data() + pos, n);
        pos += n;
        return true;
    }
    // the next section, which must carry `tag`; its bytes are [*at, *at + *n)
    bool section(uint32_t tag, const char **at, size_t *n) {
        uint32_t t = 0, z = 0;
        uint64_t nb = 0;
        if (!take(&t, 4) || !take(&z, 4) || !take(&nb, 8) || t != tag || pos + nb > buf.size()) return false;
        *at = buf.data() + pos;
        *n = (size_t)nb;
        pos += (size_t)nb;
        return true;
    }
};

bool read_file(const char *path, std::vector<char> &out) {
    FILE *f = std::fopen(path, "rb");
    if (!f) return false;
    bool ok = std::fseek(f, 0, SEEK_END) == 0;
    long sz = ok ? std::ftell(f) : -1;
    ok = ok && sz >= 0 && std::fseek(f, 0, SEEK_SET) == 0;
    if (ok) {
        out.resize((size_t)sz);
        ok = sz == 0 || std::fread(out.data(), 1, (size_t)sz, f) == (size_t)sz;
    }
    std::fclose(f);
    return ok;
}

we_status read_header(const std::vector<char> &buf, Header &h) {
    if (buf.size() < sizeof(Header)) return we_fail(WE_EINVAL, "checkpoint: file too short");
    std::memcpy(&h, buf.data(), sizeof h);
    if (std::memcmp(h.magic, kMagic, 8) != 0) return we_fail(WE_EINVAL, "checkpoint: bad magic");
    if (h.version != kVersion || h.header_bytes != sizeof(Header))
        return we_fail(WE_EINVAL, "checkpoint: unsupported version " + std::to_string(h.version));
    return WE_OK;
}

// Parse the PARM section that follows the header.
we_status read_params(Reader &rd, ParamsRec &pr) {
    const char *at;
    size_t n;
    if (!rd.section(T_PARM, &at, &n) || n != sizeof(ParamsRec)) return we_fail(WE_EINVAL, "checkpoint: bad PARM");
    std::memcpy(&pr, at, sizeof pr);
    return WE_OK;
}

template <class T>
bool slice(const char *&at, size_t &left, std::vector<T> &out, size_t count) {
    const size_t nb = count * sizeof(T);
    if (nb > left) return false;
    out.resize(count);
    if (nb) std::memcpy(out.data(), at, nb);
    at += nb;
    left -= nb;
    return true;
}

}  // namespace

extern "C" we_status we_save(we_sim *s, const char *path) {
    if (!s || !path) return we_fail(WE_EINVAL, "NULL argument");
    we_status st = we_read_err(s);   // synchronizes the stream; reports latched faults
    if (st != WE_OK) return st;
    const SimConfig &cf = s->cfg;
    Header h{};
    std::memcpy(h.magic, kMagic, 8);
    h.version = kVersion;
    h.header_bytes = sizeof(Header);
    h.S = s->S; h.R = s->net->R; h.n_runs = s->n_runs; h.NB = s->NB; h.M = s->M;
    h.max_iters = s->max_iters; h.iter = s->iter; h.cur = s->cur;
    h.net_fp = network_fingerprint(s->net);
    h.ws_bytes = cf.ws_bytes;

    ParamsRec pr{};
    pr.tau = cf.p.tau; pr.tgt_thr = cf.p.tgt_thr; pr.leap_eps = cf.p.leap_eps;
    pr.m_targ = cf.p.m_targ; pr.n_runs = cf.p.n_runs; pr.max_iters = cf.p.max_iters; pr.kernel = s->kernel;
    pr.recycle = cf.p.recycle; pr.hist_species = cf.p.hist_species; pr.hist_lo = cf.p.hist_lo;
    pr.hist_hi = cf.p.hist_hi; pr.n_joint = cf.p.n_joint; pr.joint_bins = cf.p.joint_bins;
    pr.joint_width = cf.p.joint_width; pr.record_iters = cf.p.record_iters; pr.rw_period = cf.p.rw_period;
    pr.rw_reset = cf.p.rw_reset; pr.engine = cf.p.engine; pr.resample_rule = cf.p.resample_rule;
    pr.walkers_per_wave = s->kernel == WE_KERNEL_GROUP ? 64 / s->group_lanes : 0;
    pr.n_bins = cf.n_bins; pr.n_bins2 = cf.n_bins2; pr.hist_iters = s->hist_iters;

    Writer w;
    w.raw(&h, sizeof h);
    w.section(T_PARM, &pr, sizeof pr);
    std::vector<double> grid(cf.coef);
    grid.insert(grid.end(), cf.edges.begin(), cf.edges.end());
    grid.insert(grid.end(), cf.coef2.begin(), cf.coef2.end());
    grid.insert(grid.end(), cf.edges2.begin(), cf.edges2.end());
    w.section_vec(T_GRID, grid);
    Writer arrs;
    arrs.raw(cf.tgt_coef.data(), 8 * cf.tgt_coef.size());
    arrs.raw(cf.seeds.data(), 8 * cf.seeds.size());
    arrs.raw(cf.x0.data(), 4 * cf.x0.size());
    arrs.raw(cf.x_rec.data(), 4 * cf.x_rec.size());
    arrs.raw(cf.joint.data(), 4 * cf.joint.size());
    w.section_vec(T_ARRS, arrs.buf);
    std::vector<char> ws(cf.ws_bytes);
    HIP_TRY(hipMemcpy(ws.data(), s->ws, cf.ws_bytes, hipMemcpyDeviceToHost));
    w.section_vec(T_WORK, ws);
    w.section_vec(T_NWLK, s->n_host);
    CommittorHost ch;
    st = committor_export(s, ch);
    if (st != WE_OK) return st;
    Writer cm;
    const int32_t flags[4] = {ch.trained ? 1 : 0, ch.active ? 1 : 0, ch.n_in, ch.n_qbins};
    cm.raw(flags, sizeof flags);
    if (ch.trained) {
        cm.raw(ch.params.data(), 4 * ch.params.size());
        cm.raw(ch.adam_m.data(), 4 * ch.adam_m.size());
        cm.raw(ch.adam_v.data(), 4 * ch.adam_v.size());
        cm.raw(ch.feat.data(), 4 * ch.feat.size());
        cm.raw(ch.qedges.data(), 8 * ch.qedges.size());
        cm.raw(ch.wt.data(), 4 * ch.wt.size());
    }
    w.section_vec(T_CMTR, cm.buf);

    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return we_fail(WE_EDEVICE, std::string("checkpoint: cannot open ") + tmp);
    const bool ok = std::fwrite(w.buf.data(), 1, w.buf.size(), f) == w.buf.size();
    const bool closed = std::fclose(f) == 0;
    if (!ok || !closed || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return we_fail(WE_EDEVICE, std::string("checkpoint: cannot write ") + path);
    }
    return WE_OK;
}

extern "C" we_status we_checkpoint_inspect(const char *path, we_checkpoint_info *info) {
    if (!path || !info) return we_fail(WE_EINVAL, "NULL argument");
    Reader rd;
    if (!read_file(path, rd.buf)) return we_fail(WE_EINVAL, std::string("checkpoint: cannot read ") + path);
    Header h;
    we_status st = read_header(rd.buf, h);
    if (st != WE_OK) return st;
    rd.pos = sizeof(Header);
    ParamsRec pr;
    st = read_params(rd, pr);
    if (st != WE_OK) return st;
    *info = we_checkpoint_info{};
    info->version = (int32_t)h.version;
    info->n_species = h.S; info->n_reactions = h.R; info->n_runs = h.n_runs; info->n_bins = h.NB;
    info->m_targ = h.M; info->max_iters = h.max_iters; info->iteration = h.iter;
    info->hist_lo = pr.hist_lo; info->hist_hi = pr.hist_hi; info->n_joint = pr.n_joint;
    info->joint_bins = pr.joint_bins; info->kernel = pr.kernel; info->tau = pr.tau;
    info->workspace_bytes = h.ws_bytes;
    return WE_OK;
}

extern "C" we_status we_load(const we_network *net, const char *path, void *hip_stream, void *workspace,
                             size_t workspace_bytes, we_sim **out) {
    if (!net || !path || !out) return we_fail(WE_EINVAL, "NULL argument");
    *out = nullptr;
    Reader rd;
    if (!read_file(path, rd.buf)) return we_fail(WE_EINVAL, std::string("checkpoint: cannot read ") + path);
    Header h;
    we_status st = read_header(rd.buf, h);
    if (st != WE_OK) return st;
    if (h.S != net->S || h.R != net->R || h.net_fp != network_fingerprint(net))
        return we_fail(WE_EINVAL, "checkpoint: saved with a different network");
    rd.pos = sizeof(Header);
    ParamsRec pr;
    st = read_params(rd, pr);
    if (st != WE_OK) return st;
    const int32_t S = h.S, n2 = pr.n_bins2 > 1 ? pr.n_bins2 : 0;
    if (pr.n_runs != h.n_runs || pr.n_bins < 1 || pr.n_runs < 1 || pr.n_joint < 0 || pr.n_joint > 5)
        return we_fail(WE_EINVAL, "checkpoint: inconsistent sizes");

    const char *at;
    size_t left;
    std::vector<double> coef, edges, coef2, edges2, tgt;
    std::vector<uint64_t> seeds;
    std::vector<int32_t> x0, xrec, joint, nwalk;
    if (!rd.section(T_GRID, &at, &left) || !slice(at, left, coef, S) || !slice(at, left, edges, pr.n_bins + 1) ||
        !slice(at, left, coef2, n2 ? S : 0) || !slice(at, left, edges2, n2 ? n2 + 1 : 0) || left != 0)
        return we_fail(WE_EINVAL, "checkpoint: bad GRID");
    if (!rd.section(T_ARRS, &at, &left) || !slice(at, left, tgt, S) || !slice(at, left, seeds, h.n_runs) ||
        !slice(at, left, x0, S) || !slice(at, left, xrec, S) || !slice(at, left, joint, pr.n_joint) || left != 0)
        return we_fail(WE_EINVAL, "checkpoint: bad ARRS");
    const char *ws_at;
    size_t ws_n;
    if (!rd.section(T_WORK, &ws_at, &ws_n) || ws_n != h.ws_bytes) return we_fail(WE_EINVAL, "checkpoint: bad WORK");
    if (!rd.section(T_NWLK, &at, &left) || !slice(at, left, nwalk, h.n_runs) || left != 0)
        return we_fail(WE_EINVAL, "checkpoint: bad NWLK");
    CommittorHost ch;
    if (!rd.section(T_CMTR, &at, &left)) return we_fail(WE_EINVAL, "checkpoint: bad CMTR");
    int32_t flags[4] = {0, 0, 0, 0};
    if (left < sizeof flags) return we_fail(WE_EINVAL, "checkpoint: bad CMTR");
    std::memcpy(flags, at, sizeof flags);
    at += sizeof flags;
    left -= sizeof flags;
    ch.trained = flags[0] != 0;
    ch.active = flags[1] != 0;
    ch.n_in = flags[2];
    ch.n_qbins = flags[3];
    if (ch.trained) {
        if (ch.n_in != S || ch.n_qbins != h.NB) return we_fail(WE_EINVAL, "checkpoint: bad CMTR");
        const size_t np = (size_t)(64 * ch.n_in + 64 + 64 * 64 + 64 + 64 + 1);
        const size_t nwt = (size_t)64 * ch.n_in + 64 * 64;
        if (!slice(at, left, ch.params, np) || !slice(at, left, ch.adam_m, np) || !slice(at, left, ch.adam_v, np) ||
            !slice(at, left, ch.feat, 2 * (size_t)ch.n_in) || !slice(at, left, ch.qedges, (size_t)ch.n_qbins + 1) ||
            !slice(at, left, ch.wt, nwt))
            return we_fail(WE_EINVAL, "checkpoint: bad CMTR");
    }
    if (left != 0) return we_fail(WE_EINVAL, "checkpoint: bad CMTR");

    we_grid g{};
    g.n_bins = pr.n_bins;
    g.coef = coef.data();
    g.edges = edges.data();
    g.n_bins2 = pr.n_bins2;
    g.coef2 = n2 ? coef2.data() : nullptr;
    g.edges2 = n2 ? edges2.data() : nullptr;
    we_params p{};
    p.tau = pr.tau; p.m_targ = pr.m_targ; p.n_runs = pr.n_runs; p.max_iters = pr.max_iters; p.kernel = pr.kernel;
    p.seeds = seeds.data(); p.x0 = x0.data(); p.recycle = pr.recycle; p.tgt_coef = tgt.data();
    p.tgt_thr = pr.tgt_thr; p.x_rec = xrec.data(); p.hist_species = pr.hist_species; p.hist_lo = pr.hist_lo;
    p.hist_hi = pr.hist_hi; p.n_joint = pr.n_joint; p.joint_species = pr.n_joint ? joint.data() : nullptr;
    p.joint_bins = pr.joint_bins; p.joint_width = pr.joint_width; p.record_iters = pr.record_iters;
    p.rw_period = pr.rw_period; p.rw_reset = pr.rw_reset; p.engine = pr.engine; p.leap_eps = pr.leap_eps;
    p.resample_rule = pr.resample_rule;
    p.walkers_per_wave = pr.walkers_per_wave;
    if (workspace && workspace_bytes < h.ws_bytes) return we_fail(WE_EINVAL, "checkpoint: workspace too small");

    we_sim *s = nullptr;
    st = we_init(net, &g, &p, hip_stream, workspace, workspace_bytes, &s);
    if (st != WE_OK) return st;
    if (s->cfg.ws_bytes != h.ws_bytes || s->kernel != pr.kernel) {
        we_destroy(s);
        return we_fail(WE_EINVAL, "checkpoint: the sim rebuilt from it has another layout");
    }
    hipError_t e = hipMemcpyAsync(s->ws, ws_at, ws_n, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        we_destroy(s);
        return we_hip_fail(e, "checkpoint: workspace upload");
    }
    s->iter = h.iter;
    s->cur = h.cur;
    s->hist_iters = pr.hist_iters;
    s->n_host = nwalk;
    st = committor_import(s, ch);
    if (st != WE_OK) {
        we_destroy(s);
        return st;
    }
    *out = s;
    return WE_OK;
}
