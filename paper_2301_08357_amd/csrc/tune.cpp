// Autotuners for the launch shapes of the pressure solver.
//
// Both tuners time short runs of the real CG iterations on the caller's own
// operators (a right-hand side of ones, a tolerance no run can reach, so
// every candidate runs the same number of iterations) and keep the fastest
// candidate.  Choices are cached in a plain text file, one line per choice:
//     <key, 16 hex digits> <value 0> <value 1> <ms per iteration>
// The key hashes (FNV-1a, 64 bit) the tuner's name, the device (architecture
// name and compute-unit count), the library build and the sizes of the
// meshes, so a rebuilt library or another device tunes again.

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pressure_cg.h"

namespace {

constexpr double TUNE_RTOL = 1e-300;   // never met within a tuning run

struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void bytes(const void *p, size_t n)
    {
        const unsigned char *c = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; ++i) {
            h ^= c[i];
            h *= 1099511628211ull;
        }
    }
    void str(const char *s) { bytes(s, std::strlen(s) + 1); }
    void i64(int64_t v) { bytes(&v, sizeof v); }
};

int device_key(Fnv &f)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PM_EHIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return PM_EHIP;
    f.str(prop.gcnArchName);
    f.i64(prop.multiProcessorCount);
    f.str(__DATE__ " " __TIME__);   // the library build
    return PM_OK;
}

bool cache_lookup(const char *path, uint64_t key, int32_t v[2], double *ms)
{
    if (!path) return false;
    FILE *fp = std::fopen(path, "r");
    if (!fp) return false;
    char line[256];
    bool found = false;
    while (std::fgets(line, sizeof line, fp)) {
        unsigned long long k = 0;
        int a = 0, b = 0;
        double t = 0.0;
        if (std::sscanf(line, "%llx %d %d %lf", &k, &a, &b, &t) == 4 && k == key) {
            v[0] = a;
            v[1] = b;
            *ms = t;
            found = true;   // the last line for a key wins
        }
    }
    std::fclose(fp);
    return found;
}

void cache_store(const char *path, uint64_t key, const int32_t v[2], double ms)
{
    if (!path) return;
    FILE *fp = std::fopen(path, "a");
    if (!fp) return;
    std::fprintf(fp, "%016llx %d %d %.6g\n", (unsigned long long)key, v[0], v[1], ms);
    std::fclose(fp);
}

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// device vector of n ones
int ones(int64_t n, double **out)
{
    *out = nullptr;
    if (hipMalloc((void **)out, sizeof(double) * size_t(n)) != hipSuccess) return PM_ENOMEM;
    std::vector<double> h(size_t(n), 1.0);
    if (hipMemcpy(*out, h.data(), sizeof(double) * size_t(n), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(*out);
        *out = nullptr;
        return PM_EHIP;
    }
    return PM_OK;
}

// Time per CG iteration of one batch shape: every mesh starts a solve, one
// warm-up step, then `steps` timed steps (each a graph replay of 16
// iterations plus the host's status read, as in a real batched solve).
int time_batch(pm_handle *const *hs, int32_t n, const int32_t params[3], int steps, const double *rhs,
               double *p, double *ms_per_iter)
{
    pm_batch *b = nullptr;
    int st = pressure_batch_create(hs, n, params, &b);
    if (st != PM_OK) return st;
    const int max_iter = (steps + 2) * 16 + 2;
    for (int m = 0; m < n && st == PM_OK; ++m) st = pressure_batch_begin(b, m, rhs, nullptr, TUNE_RTOL, max_iter, nullptr);
    std::vector<int32_t> done(size_t(n), 0);
    if (st == PM_OK) st = pressure_batch_step(b, done.data(), nullptr);
    const double t0 = now_ms();
    for (int k = 0; k < steps && st == PM_OK; ++k) st = pressure_batch_step(b, done.data(), nullptr);
    const double t1 = now_ms();
    // leave every handle idle: finish the solves (their results are discarded)
    for (int m = 0; m < n; ++m) {
        if (st != PM_OK) break;
        int32_t it = 0;
        double rel = 0.0;
        // run the remaining iterations of each solve to its max_iter
        while (!done[m] && st == PM_OK) st = pressure_batch_step(b, done.data(), nullptr);
        if (st == PM_OK) {
            const int c = pressure_batch_finish(b, m, rhs, TUNE_RTOL, p, &it, &rel, nullptr);
            if (c < 0 && c != PM_EBREAKDOWN) st = c;
        }
    }
    pressure_batch_destroy(b);
    if (st == PM_OK) *ms_per_iter = (t1 - t0) / (16.0 * steps);
    return st;
}

}  // namespace

extern "C" {

int pressure_batch_tune(pm_handle *const *handles, int32_t n, int32_t iters, const char *cache_path,
                        int32_t *params_out, double *ms_per_iter)
{
    if (!handles || n < 1 || iters < 1 || !params_out || !ms_per_iter) return PM_EINVAL;
    Fnv f;
    f.str("batch-shape");
    int st = device_key(f);
    if (st != PM_OK) return st;
    f.i64(n);
    int64_t n_max = 0;
    for (int m = 0; m < n; ++m) {
        if (!handles[m]) return PM_EINVAL;
        int64_t info[8];
        st = pressure_info(handles[m], info, 8);
        if (st != PM_OK) return st;
        for (int k : {0, 1, 3, 6, 7}) f.i64(info[k]);   // N, E, dim, tiles, instances
        n_max = std::max<int64_t>(n_max, info[0]);
    }
    int32_t v[2];
    double ms = 0.0;
    if (cache_lookup(cache_path, f.h, v, &ms)) {
        params_out[0] = v[0];
        params_out[1] = v[1];
        *ms_per_iter = ms;
        return PM_OK;
    }
    double *rhs = nullptr, *p = nullptr;
    st = ones(n_max, &rhs);
    if (st == PM_OK) st = ones(n_max, &p);
    const int steps = std::max(1, (iters + 15) / 16);
    double best = 0.0;
    int32_t best_v[2] = {0, 0};
    for (int32_t tps : {1, 2, 4, 8}) {
        for (int32_t npl : {2, 4, 8, 16}) {
            if (st != PM_OK) break;
            const int32_t params[3] = {tps, npl, 1};
            double t = 0.0;
            st = time_batch(handles, n, params, steps, rhs, p, &t);
            if (st == PM_OK && (best_v[0] == 0 || t < best)) {
                best = t;
                best_v[0] = tps;
                best_v[1] = npl;
            }
        }
    }
    if (rhs) (void)hipFree(rhs);
    if (p) (void)hipFree(p);
    if (st != PM_OK) return st;
    params_out[0] = best_v[0];
    params_out[1] = best_v[1];
    *ms_per_iter = best;
    cache_store(cache_path, f.h, best_v, best);
    return PM_OK;
}

int pressure_tune_tile(const pm_mesh *mesh, const double *elem_coef, double mass_coef, double dt, int32_t flags,
                       int32_t iters, const char *cache_path, int32_t *flags_out, double *ms_per_iter)
{
    if (!mesh || !elem_coef || iters < 1 || !flags_out || !ms_per_iter) return PM_EINVAL;
    const int32_t base = flags & ~PM_TILE_MASK;
    Fnv f;
    f.str("tile-size");
    int st = device_key(f);
    if (st != PM_OK) return st;
    f.i64(mesh->dim);
    f.i64(mesh->n_nodes);
    f.i64(mesh->n_elems);
    f.i64(base);
    int32_t v[2];
    double ms = 0.0;
    if (cache_lookup(cache_path, f.h, v, &ms)) {
        *flags_out = base | v[0];
        *ms_per_iter = ms;
        return PM_OK;
    }
    double *rhs = nullptr, *p = nullptr;
    st = ones(mesh->n_nodes, &rhs);
    if (st == PM_OK) st = ones(mesh->n_nodes, &p);
    double best = 0.0;
    int32_t best_tile = 0;
    for (int32_t tile : {PM_TILE_128, PM_TILE_256, PM_TILE_512}) {
        if (st != PM_OK) break;
        pm_handle *h = nullptr;
        const int s = pressure_setup(mesh, elem_coef, mass_coef, dt, base | tile, &h);
        if (s == PM_EINVAL) continue;   // this tile size's tables do not fit the LDS
        if (s != PM_OK) {
            st = s;
            break;
        }
        int32_t it = 0;
        double rel = 0.0;
        // warm-up, then the timed run
        int c = pressure_solve(h, rhs, nullptr, TUNE_RTOL, 8, p, &it, nullptr, &rel, nullptr);
        double t = 0.0;
        if (c >= 0 || c == PM_EBREAKDOWN) {
            const double t0 = now_ms();
            c = pressure_solve(h, rhs, nullptr, TUNE_RTOL, iters, p, &it, nullptr, &rel, nullptr);
            t = (now_ms() - t0) / std::max(1, int(it));
        }
        pressure_destroy(h);
        if (c < 0 && c != PM_EBREAKDOWN) {
            st = c;
            break;
        }
        if (best_tile == 0 || t < best) {
            best = t;
            best_tile = tile;
        }
    }
    if (rhs) (void)hipFree(rhs);
    if (p) (void)hipFree(p);
    if (st != PM_OK) return st;
    if (best_tile == 0) return PM_EINVAL;
    v[0] = best_tile;
    v[1] = 0;
    *flags_out = base | best_tile;
    *ms_per_iter = best;
    cache_store(cache_path, f.h, v, best);
    return PM_OK;
}

}  // extern "C"
