// Host runtime: geometry, device memory, pointer classification, event timing and the
// launch-configuration autotuner.
#include "runtime.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

namespace wl {

static thread_local std::string g_last_error;

void set_last_error(const std::string &m) { g_last_error = m; }
const std::string &last_error() { return g_last_error; }

void hip_fail(hipError_t e, const char *what, const char *file, int line) {
    std::ostringstream os;
    os << "HIP error " << hipGetErrorName(e) << " (" << hipGetErrorString(e) << ") in " << what << " at " << file
       << ":" << line;
    throw Error(e == hipErrorOutOfMemory ? WILSON_OUT_OF_MEMORY : WILSON_DEVICE_ERROR, os.str());
}

Geom make_geom(const int32_t dims[4]) {
    Geom g;
    for (int k = 0; k < 4; k++) g.L[k] = dims[k];
    g.Lxh = dims[0] / 2;
    const long long V = (long long)dims[0] * dims[1] * dims[2] * dims[3];
    g.Vh = (int)(V / 2);
    g.stride = (int)(((V / 2) + 63) / 64 * 64);
    g.sy = g.Lxh;
    g.sz = g.Lxh * dims[1];
    g.st = g.Lxh * dims[1] * dims[2];
    g.dLxh = make_fastdiv((uint32_t)g.Lxh);
    g.dLy = make_fastdiv((uint32_t)dims[1]);
    g.dLz = make_fastdiv((uint32_t)dims[2]);
    // the multiply-high division is exact for every n < 2^31; spot-check the sizes in use
    for (const FastDiv *f : {&g.dLxh, &g.dLy, &g.dLz})
        for (uint32_t n : {0u, 1u, f->d - 1, f->d, (uint32_t)g.Vh - 1, (uint32_t)g.Vh, 0x7fffffffu})
            if (fdiv(n, *f) != n / f->d) throw Error(WILSON_INVALID_ARG, "index division self-check failed");
    return g;
}

void DevBuf::alloc(size_t bytes) {
    release();
    if (bytes == 0) return;
    hipError_t e = hipMalloc(&p_, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        p_ = nullptr;
        throw Error(WILSON_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    n_ = bytes;
}

void DevBuf::release() {
    if (p_) (void)hipFree(p_);
    p_ = nullptr;
    n_ = 0;
}

void PinnedBuf::alloc(size_t bytes) {
    if (h_) (void)hipHostFree(h_);
    h_ = d_ = nullptr;
    n_ = 0;
    WL_HIP(hipHostMalloc(&h_, bytes, hipHostMallocMapped | hipHostMallocCoherent));
    WL_HIP(hipHostGetDevicePointer(&d_, h_, 0));
    std::memset(h_, 0, bytes);
    n_ = bytes;
}

PinnedBuf::~PinnedBuf() {
    if (h_) (void)hipHostFree(h_);
}

void SolveHostRes::create(int nrhs) {
    mirror.alloc(sizeof(RhsState) * nrhs * kStateRing);
    hinit.alloc(sizeof(RhsState) * nrhs);
    hread.alloc(sizeof(RhsState) * nrhs);
    for (auto &e : ring) WL_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    cap = nrhs;
}

SolveHostRes::~SolveHostRes() {
    for (auto &e : ring)
        if (e) (void)hipEventDestroy(e);
}

bool is_device_ptr(const void *p) {
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

size_t partials_doubles(const Geom &g, int nrhs) {
    const size_t hop_nb = (size_t)(g.Vh + 63) / 64 * 2;  // smallest hop tile; x2: both parities in one row
    size_t nb = hop_nb;
    for (int p : {P64, P32, P16}) nb = std::max(nb, (size_t)blas_nblocks(g, p));
    return (size_t)nrhs * 3 * nb + 64;
}

double hop_bytes(const HopArgs &a) {
    const double sb = 24.0 * real_bytes(a.in.prec) + (a.in.prec == P16 ? 4.0 : 0.0);
    const double lb = 8.0 * 18.0 * real_bytes(a.gprec);  // algorithmic: a link is 18 reals
    double per_rhs = sb;                 // input field, each site once
    if (!a.nostore) per_rhs += sb;       // output
    if (a.has_y) per_rhs += sb;
    if (a.has_z) per_rhs += sb;
    if (a.red == RED_DOT) per_rhs += sb;  // dot partner
    // clover site blocks: 72 reals per site, read once for all right-hand sides
    const double cb = a.clov_mode != CLV_NONE ? kClovReals * real_bytes(a.in.prec == P64 ? P64 : P32) : 0.0;
    return (double)a.g.Vh * (lb + cb + a.nrhs * per_rhs);
}

}  // namespace wl

using namespace wl;

hipEvent_t wilson_ctx::get_event() {
    if (!event_pool.empty()) {
        hipEvent_t e = event_pool.back();
        event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    WL_HIP(hipEventCreate(&e));
    return e;
}

void wilson_ctx::drain_timing() {
    for (auto &p : pending) {
        WL_HIP(hipEventSynchronize(p.b));
        float ms = 0.f;
        WL_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        t_ms[p.cls] += ms;
        launches[p.cls] += 1;
        t_bytes[p.cls] += p.bytes;
        event_pool.push_back(p.a);
        event_pool.push_back(p.b);
    }
    pending.clear();
}

void *wilson_ctx::stage(DevBuf &b, size_t bytes) {
    if (b.size() < bytes) {
        WL_HIP(hipStreamSynchronize(stream));
        b.alloc(bytes);
    }
    return b.get();
}

TuneTable &tune_table() {
    static TuneTable *t = [] {
        TuneTable *T = new TuneTable();  // lives until the process ends
        const char *env = std::getenv("WILSON_TUNE");
        if (env && std::strcmp(env, "0") == 0) T->enabled = false;
        const char *path = std::getenv("WILSON_TUNE_CACHE");
        if (!path || !*path) return T;
        T->path = path;
        std::ifstream in(T->path);
        std::string line;
        // one JSON object per line: {"key": "...", "block": B, "rpt": R, "xcd": X, "zblk": Z, "lds_kb": K,
        // "wsplit": W, "shx": S, "dsplit": D, "ldsl": K, "tm": M, "ms": T}
        while (std::getline(in, line)) {
            const size_t k0 = line.find("\"key\": \"");
            if (k0 == std::string::npos) continue;
            const size_t k1 = line.find('"', k0 + 8);
            if (k1 == std::string::npos) continue;
            const std::string key = line.substr(k0 + 8, k1 - k0 - 8);
            wl::LaunchCfg c;
            if (std::sscanf(line.c_str() + k1,
                            "\", \"block\": %d, \"rpt\": %d, \"xcd\": %d, \"zblk\": %d, \"lds_kb\": %d, \"wsplit\": %d, "
                            "\"shx\": %d, \"dsplit\": %d, \"ldsl\": %d, \"tm\": %d",
                            &c.block, &c.rpt, &c.xcd, &c.zblk, &c.lds_kb, &c.wsplit, &c.shx, &c.dsplit, &c.ldsl,
                            &c.tm) >= 5)
                T->cfg[key] = c;
        }
        return T;
    }();
    return *t;
}

void TuneTable::save(const std::string &key, const wl::LaunchCfg &c, double ms) {
    if (path.empty()) return;
    std::ofstream out(path, std::ios::app);
    out << "{\"key\": \"" << key << "\", \"block\": " << c.block << ", \"rpt\": " << c.rpt << ", \"xcd\": " << c.xcd
        << ", \"zblk\": " << c.zblk << ", \"lds_kb\": " << c.lds_kb << ", \"wsplit\": " << c.wsplit
        << ", \"shx\": " << c.shx << ", \"dsplit\": " << c.dsplit << ", \"ldsl\": " << c.ldsl << ", \"tm\": " << c.tm
        << ", \"ms\": " << ms
        << "}\n";
}

namespace wl {

// Launches are tuned per lattice, precision pair, link storage and class of RHS count
// (1, 2, 3-4, 5-8, 9+), not per epilogue or exact count: the best shape depends on the
// streams, not on a fused dot or an added vector, and a finer key would re-tune for every
// request size a server sees.
static int rhs_class(int n) { return n <= 2 ? n : (n <= 4 ? 4 : (n <= 8 ? 8 : 12)); }

static std::string hop_key(const HopArgs &a) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::ostringstream os;
    os << "dev=" << dev << " hop sp=" << a.in.prec << " gp=" << a.gprec << " rc=" << a.recon << " rhs=" << rhs_class(a.nrhs)
       << " dims=" << a.g.L[0] << "x" << a.g.L[1] << "x" << a.g.L[2] << "x" << a.g.L[3];
    return os.str();
}

// A configuration made valid for this launch: the RHS split shrinks to a divisor of nrhs,
// then the plane blocking, the wave split and the block size fall back if they still do not fit.
static LaunchCfg fit_cfg(const HopArgs &a, LaunchCfg c) {
    if (hop_cfg_valid(a, c)) return c;
    if (c.dsplit) {  // the direction split's shape is fixed; otherwise the default block
        c.dsplit = 0;
        c.block = 256;
    }
    if (c.tm && !hop_cfg_valid(a, c)) c.tm = 0;
    if (c.ldsl && !hop_cfg_valid(a, c)) c.ldsl = 0;
    if (a.clov_mode != CLV_NONE) {
        c.rpt = 1;
        c.shx = 0;
    }
    while (c.rpt > 1 && (a.nrhs % c.rpt || (a.in.prec == P64 && c.rpt > 2) || c.shx)) c.rpt--;
    if (c.zblk > 0 && a.g.L[2] % c.zblk) c.zblk = 0;
    if (!hop_cfg_valid(a, c)) c.wsplit = 0;
    if (!hop_cfg_valid(a, c)) c.block = 256;
    if (!hop_cfg_valid(a, c)) c.rpt = 1;
    return c;
}

// Lattices below 4096 sites per parity are not tuned: they take the direction split (the
// plain kernel would run a few dozen waves, each a chain of dependent gathers).
static LaunchCfg default_cfg(const HopArgs &a) {
    LaunchCfg c;
    c.xcd = 1;
    if (a.g.Vh < 4096) {
        c.block = 320;
        c.dsplit = 1;
        if (hop_cfg_valid(a, c)) return c;
        c.dsplit = 0;
    }
    c.block = 256;
    const int maxr = a.in.prec == P64 ? 2 : 4;
    for (int r = maxr; r >= 1; r--)
        if (a.nrhs % r == 0) { c.rpt = r; break; }
    return c;
}

// Time each candidate configuration on the live arguments (the hop is a pure function of
// its inputs, so repeated launches are harmless) and keep the fastest.
static LaunchCfg tune_hop(wilson_ctx *ctx, const HopArgs &a, double *best_ms) {
    std::vector<LaunchCfg> cands;
    // plain block order once (the XCD-contiguous order has won every measured case), then
    // the XCD order over block size, RHS split, plane blocking, LDS cap and wave split
    {
        LaunchCfg c = default_cfg(a);
        c.xcd = 0;
        cands.push_back(c);
    }
    // plane blocks of 4 and 8 z-planes, and of Lz/8: with the XCD-contiguous block order that
    // one gives each of the 8 XCDs one z-range through every t-slice
    std::vector<int> zblks = {0, 4, 8};
    if (a.g.L[2] % 8 == 0 && a.g.L[2] / 8 != 4 && a.g.L[2] / 8 != 8) zblks.push_back(a.g.L[2] / 8);
    for (int shx : {0, 1})
        for (int wsplit : {0, 1})
            for (int block : {64, 128, 192, 256})
                for (int rpt : {1, 2, 3, 4})
                    for (int zblk : zblks)
                        for (int lds_kb : {0, 40}) {
                            if (wsplit && a.nrhs == 1) continue;
                            LaunchCfg c;
                            c.block = block;
                            c.rpt = rpt;
                            c.xcd = 1;
                            c.zblk = zblk;
                            c.lds_kb = lds_kb;
                            c.wsplit = wsplit;
                            c.shx = shx;
                            if (hop_cfg_valid(a, c)) cands.push_back(c);
                        }
    for (int ldsl : {1, 2})  // the wave split with the tile's links in LDS (2: rebuilt to full links)
        for (int block : {128, 192, 256})
            for (int rpt : {1, 2})
                for (int shx : {0, 1})
                    for (int zblk : zblks) {
                        LaunchCfg c;
                        c.block = block;
                        c.rpt = rpt;
                        c.zblk = zblk;
                        c.wsplit = 1;
                        c.shx = shx;
                        c.ldsl = ldsl;
                        if (a.nrhs > 1 && hop_cfg_valid(a, c)) cands.push_back(c);
                    }
    // t-marching over 2, 4 or 8 slices: direct links (one or all RHS groups per block) or, with
    // the wave split, links staged in LDS per step
    for (int tm : {2, 4, 8})
        for (int wsplit : {0, 1})
            for (int ldsl : {0, 1})
                for (int shx : {0, 1})
                    for (int block : {64, 128, 192, 256})
                        for (int rpt : {1, 2, 3, 4}) {
                            if (ldsl && !wsplit) continue;
                            if (wsplit && a.nrhs == 1) continue;
                            LaunchCfg c;
                            c.block = block;
                            c.rpt = rpt;
                            c.wsplit = wsplit;
                            c.ldsl = ldsl;
                            c.shx = shx;
                            c.tm = tm;
                            if (hop_cfg_valid(a, c)) cands.push_back(c);
                        }
    for (int xcd : {1, 0}) {  // the direction split (small lattices)
        LaunchCfg c;
        c.block = 320;
        c.xcd = xcd;
        c.dsplit = 1;
        if (hop_cfg_valid(a, c)) cands.push_back(c);
    }
    hipEvent_t e0, e1;
    WL_HIP(hipEventCreate(&e0));
    WL_HIP(hipEventCreate(&e1));
    const bool verbose = std::getenv("WILSON_TUNE_VERBOSE") != nullptr;
    auto time_cfg = [&](const LaunchCfg &c, int reps) {
        WL_HIP(hipEventRecord(e0, ctx->stream));
        for (int r = 0; r < reps; r++) WL_HIP(launch_hop(a, c, ctx->stream));
        WL_HIP(hipEventRecord(e1, ctx->stream));
        WL_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        WL_HIP(hipEventElapsedTime(&ms, e0, e1));
        return (double)ms / reps;
    };
    // first pass: every candidate briefly
    const int reps = a.g.Vh >= (1 << 18) ? 3 : 10;
    std::vector<std::pair<double, LaunchCfg>> timed;
    for (const auto &c : cands) {
        if (launch_hop(a, c, ctx->stream) != hipSuccess) {  // warm-up; skip shapes that cannot launch
            (void)hipGetLastError();
            continue;
        }
        const double per = time_cfg(c, reps);
        if (verbose)
            std::fprintf(stderr, "[tune] %s block=%d rpt=%d xcd=%d zblk=%d lds=%d ws=%d shx=%d ds=%d ll=%d tm=%d: %.2f us\n",
                         hop_key(a).c_str(), c.block, c.rpt, c.xcd, c.zblk, c.lds_kb, c.wsplit, c.shx, c.dsplit, c.ldsl,
                         c.tm, per * 1e3);
        timed.push_back({per, c});
    }
    LaunchCfg best = default_cfg(a);
    double bms = 1e30;
    if (!timed.empty()) {
        // second pass: the leading shapes, often within a few per cent of each other, again
        // in rounds that alternate between them, so that a short first timing or a drift of
        // the clock does not decide; the shape with the least total time wins
        std::stable_sort(timed.begin(), timed.end(),
                         [](const auto &x, const auto &y) { return x.first < y.first; });
        const size_t k = std::min<size_t>(timed.size(), 6);
        std::vector<double> total(k, 0.0);
        const int rounds = 3, reps2 = a.g.Vh >= (1 << 18) ? 5 : 20;
        // On large lattices a solver's next hop is of the other parity, which leaves little
        // of this hop's data in the Infinity Cache, while repeated launches of one hop find
        // part of theirs there and favour the shapes whose order profits from it.  So each
        // timed launch follows a hop of the other parity over the same links (the input
        // read as that parity's field, nothing stored, nothing reduced), not timed.
        HopArgs sa = a;
        sa.par = 1 - a.par;
        sa.has_y = sa.has_z = 0;
        sa.nostore = 1;
        sa.red = RED_NONE;
        sa.clov_mode = CLV_NONE;
        const LaunchCfg sc = default_cfg(sa);
        auto time_after_other = [&](const LaunchCfg &c, int n) {
            double sum = 0.0;
            for (int r = 0; r < n; r++) {
                WL_HIP(launch_hop(sa, sc, ctx->stream));
                WL_HIP(hipEventRecord(e0, ctx->stream));
                WL_HIP(launch_hop(a, c, ctx->stream));
                WL_HIP(hipEventRecord(e1, ctx->stream));
                WL_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                WL_HIP(hipEventElapsedTime(&ms, e0, e1));
                sum += ms;
            }
            return sum / n;
        };
        const bool cold = a.g.Vh >= (1 << 18);
        for (int round = 0; round < rounds; round++)
            for (size_t j = 0; j < k; j++)
                total[j] += cold ? time_after_other(timed[j].second, reps2) : time_cfg(timed[j].second, reps2);
        for (size_t j = 0; j < k; j++) {
            const double per = total[j] / rounds;
            if (verbose) {
                const LaunchCfg &c = timed[j].second;
                std::fprintf(stderr, "[tune] %s second pass block=%d rpt=%d xcd=%d zblk=%d lds=%d ws=%d shx=%d ds=%d ll=%d "
                             "tm=%d: %.2f us\n", hop_key(a).c_str(), c.block, c.rpt, c.xcd, c.zblk, c.lds_kb, c.wsplit,
                             c.shx, c.dsplit, c.ldsl, c.tm, per * 1e3);
            }
            if (per < bms) {
                bms = per;
                best = timed[j].second;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *best_ms = bms;
    return best;
}

int hop(wilson_ctx *ctx, HopArgs &a, double algorithmic_bytes) {
    if (a.nrhs < 1 || a.nrhs > kMaxRhs) throw Error(WILSON_INVALID_ARG, "nrhs out of range");
    if (a.out.data == a.in.data || (a.has_y && a.out.data == a.y.data) || (a.has_z && a.out.data == a.z.data))
        throw Error(WILSON_INVALID_ARG, "hop output aliases an input");
    if (a.clov_mode != CLV_NONE && a.clov == nullptr) throw Error(WILSON_INVALID_ARG, "clover blocks missing");
    if (!ctx->cfg_read) {
        ctx->cfg_read = true;
        const char *fc = std::getenv("WILSON_HOP_CFG");
        if (fc) {
            LaunchCfg &c = ctx->forced_cfg;
            ctx->forced = std::sscanf(fc, "%d,%d,%d,%d,%d,%d,%d,%d,%d,%d", &c.block, &c.rpt, &c.xcd, &c.zblk, &c.lds_kb,
                                      &c.wsplit, &c.shx, &c.dsplit, &c.ldsl, &c.tm) >= 4;
        }
    }
    LaunchCfg cfg;
    const wilson_ctx::HotKey hk = {a.in.prec, a.gprec, a.recon, rhs_class(a.nrhs), {a.g.L[0], a.g.L[1], a.g.L[2], a.g.L[3]}};
    const wilson_ctx::HotKey *found = nullptr;
    for (const auto &e : ctx->hot)
        if (e.first == hk) {
            cfg = e.second;
            found = &e.first;
            break;
        }
    if (!found) {
        bool cache = true;
        TuneTable &T = tune_table();
        const std::string key = hop_key(a);
        std::lock_guard<std::mutex> lk(T.mu);
        auto it = T.cfg.find(key);
        if (ctx->forced) {
            cfg = ctx->forced_cfg;  // the pinned shape; fitted to each launch below
        } else if (it != T.cfg.end()) {
            cfg = it->second;
        } else if (T.enabled && a.g.Vh >= 4096 && !ctx->no_tune) {
            double ms = 0;
            cfg = tune_hop(ctx, a, &ms);
            T.cfg[key] = cfg;
            T.save(key, cfg, ms);
        } else if (ctx->no_tune) {
            cfg = default_cfg(a);  // kept nowhere: a later call may still tune this shape
            cache = false;
        } else {
            cfg = default_cfg(a);
            T.cfg[key] = cfg;
        }
        if (cache && ctx->hot.size() < 32) ctx->hot.push_back({hk, cfg});
    }
    // a stored or pinned shape may not suit this launch (clover epilogue, RHS count): keep
    // its order and block, fit the RHS split
    cfg = fit_cfg(a, cfg);
    ctx->hop_launch_count++;
    ctx->bytes_issued += algorithmic_bytes;
    ctx->flops_issued += (a.clov_mode != CLV_NONE ? 1896.0 : 1320.0) * a.g.Vh * a.nrhs;
    if (ctx->timing) {
        hipEvent_t e0 = ctx->get_event(), e1 = ctx->get_event();
        WL_HIP(hipEventRecord(e0, ctx->stream));
        WL_HIP(launch_hop(a, cfg, ctx->stream));
        WL_HIP(hipEventRecord(e1, ctx->stream));
        ctx->pending.push_back({e0, e1, WILSON_KERNEL_HOP, algorithmic_bytes});
    } else {
        WL_HIP(launch_hop(a, cfg, ctx->stream));
    }
    return hop_nblocks(a, cfg);
}

void blas(wilson_ctx *ctx, int op, BlasArgs &a, double algorithmic_bytes) {
    ctx->bytes_issued += algorithmic_bytes;
    if (ctx->timing) {
        hipEvent_t e0 = ctx->get_event(), e1 = ctx->get_event();
        WL_HIP(hipEventRecord(e0, ctx->stream));
        WL_HIP(launch_blas(op, a, ctx->stream));
        WL_HIP(hipEventRecord(e1, ctx->stream));
        ctx->pending.push_back({e0, e1, WILSON_KERNEL_BLAS, algorithmic_bytes});
    } else {
        WL_HIP(launch_blas(op, a, ctx->stream));
    }
}

}  // namespace wl
