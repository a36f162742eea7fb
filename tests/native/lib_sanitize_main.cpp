// Drives the library's host code through the C ABI with
// UndefinedBehaviorSanitizer in the host code (test infrastructure: the
// library sources are compiled with the sanitizer for the host side only,
// the GPU code is the ordinary build; tests/test_gpu_host_sanitized.py runs
// it).  Covers plan creation and assembly in several modes, the plan CG, a
// mesh error, a batch built on the builder threads (and a failing one), and
// the server's worker threads.  Prints "ok" at the end; a sanitizer report
// ends the process with a nonzero status.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "nlfem.h"

namespace {

struct Mesh {
    std::vector<double> coords;
    std::vector<int32_t> tets;
    std::vector<uint8_t> vfree;
    std::vector<double> f, g;
    nlfem_mesh m{};
};

// n^3 unit cubes on [0,1]^3, six tets per cube along its main diagonal; a
// vertex is free when every coordinate lies in (delta, 1 - delta)
void kuhn(int n, double delta, Mesh& M) {
    const int p = n + 1;
    auto id = [&](int i, int j, int k) { return (int32_t)(i + p * (j + p * k)); };
    for (int k = 0; k < p; ++k)
        for (int j = 0; j < p; ++j)
            for (int i = 0; i < p; ++i) {
                const double x = (double)i / n, y = (double)j / n, z = (double)k / n;
                M.coords.insert(M.coords.end(), {x, y, z});
                const bool in = x > delta && x < 1 - delta && y > delta && y < 1 - delta && z > delta && z < 1 - delta;
                M.vfree.push_back(in ? 1 : 0);
                M.g.push_back(x * x);
            }
    const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                for (const auto& pr : perm) {
                    int c[3] = {i, j, k};
                    M.tets.push_back(id(c[0], c[1], c[2]));
                    for (int s = 0; s < 3; ++s) {
                        ++c[pr[s]];
                        M.tets.push_back(id(c[0], c[1], c[2]));
                    }
                }
    M.f.assign(M.tets.size(), -2.0);
    M.m.n_vertices = (int64_t)M.vfree.size();
    M.m.n_tets = (int64_t)(M.tets.size() / 4);
    M.m.coords = M.coords.data();
    M.m.tets = M.tets.data();
    M.m.vertex_free = M.vfree.data();
    M.m.tet_region = nullptr;
    M.m.mem_kind = 0;
}

nlfem_params params(double delta, int N) {
    nlfem_params p{};
    p.delta = delta;
    p.psi = 1.0;
    p.mc_samples = N;
    p.seed = 5;
    return p;
}

int failures = 0;
void check(bool ok, const char* what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

template <typename T>
T* dmalloc(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, (n ? n : 1) * sizeof(T)) != hipSuccess) {
        std::fprintf(stderr, "hipMalloc failed\n");
        std::exit(3);
    }
    return (T*)p;
}

// plan, assembly and plan CG of one mesh; returns the CG iteration count
int solve_one(nlfem_ctx* ctx, const Mesh& M, const nlfem_params& p) {
    nlfem_plan* plan = nullptr;
    check(nlfem_plan_create(ctx, &M.m, &p, &plan) == NLFEM_OK, "plan_create");
    if (!plan) return -1;
    int64_t nf = 0, nff = 0, nfc = 0, pc[5];
    size_t ws = 0;
    check(nlfem_plan_info(plan, &nf, &nff, &nfc, pc, &ws) == NLFEM_OK, "plan_info");
    double* f = dmalloc<double>(M.f.size());
    double* g = dmalloc<double>(M.g.size());
    hipMemcpy(f, M.f.data(), M.f.size() * 8, hipMemcpyHostToDevice);
    hipMemcpy(g, M.g.data(), M.g.size() * 8, hipMemcpyHostToDevice);
    int64_t* frp = dmalloc<int64_t>(nf + 1);
    int32_t* fcol = dmalloc<int32_t>(nff);
    double* fval = dmalloc<double>(nff);
    int64_t* crp = dmalloc<int64_t>(nf + 1);
    int32_t* ccol = dmalloc<int32_t>(nfc);
    double* cval = dmalloc<double>(nfc);
    double* rhs = dmalloc<double>(nf);
    int32_t* f2v = dmalloc<int32_t>(nf);
    double* x = dmalloc<double>(nf);
    check(nlfem_assemble(plan, f, g, frp, fcol, fval, crp, ccol, cval, rhs, f2v) == NLFEM_OK, "assemble");
    hipMemset(x, 0, (size_t)(nf ? nf : 1) * 8);
    int32_t its = 0;
    double rr = 0.0;
    const nlfem_status st = nlfem_plan_cg(plan, fval, rhs, x, 1e-10, 1000, &its, &rr);
    check(st == NLFEM_OK, "plan_cg");
    double t[6];
    check(nlfem_plan_timings(plan, t) == NLFEM_OK, "timings");
    check(nlfem_plan_destroy(plan) == NLFEM_OK, "plan_destroy");
    for (void* q : std::vector<void*>{f, g, frp, fcol, fval, crp, ccol, cval, rhs, f2v, x}) hipFree(q);
    return its;
}

}  // namespace

int main() {
    nlfem_ctx* ctx = nullptr;
    if (nlfem_create(&ctx, 0, nullptr, 0) != NLFEM_OK) {
        std::fprintf(stderr, "no context\n");
        return 3;
    }
    Mesh A;
    kuhn(6, 0.25, A);
    // single plans in four modes
    {
        nlfem_params p = params(0.25, 16);
        std::printf("fullcaps pair fp64: cg %d\n", solve_one(ctx, A, p));
        p.keying = NLFEM_KEY_ELEMENT;
        std::printf("element keying: cg %d\n", solve_one(ctx, A, p));
        p.keying = NLFEM_KEY_PAIR;
        p.cap_sampling = NLFEM_CAPS_OUTSIDE_UI;
        std::printf("cap region: cg %d\n", solve_one(ctx, A, p));
        p.cap_sampling = NLFEM_CAPS_WHOLE_ELEMENT;
        p.precision = NLFEM_FP32_LOCAL;
        p.strategy = NLFEM_NOCAPS;
        std::printf("fp32-local nocaps: cg %d\n", solve_one(ctx, A, p));
    }
    // a mesh error: a vertex index out of range
    {
        Mesh B;
        kuhn(4, 0.25, B);
        B.tets[7] = (int32_t)B.m.n_vertices + 2;
        nlfem_params p = params(0.25, 8);
        nlfem_plan* plan = nullptr;
        check(nlfem_plan_create(ctx, &B.m, &p, &plan) == NLFEM_E_MESH, "mesh error reported");
        check(plan == nullptr, "no plan after a mesh error");
    }
    // a batch of nine meshes (built on the builder threads), then a failing one
    {
        std::vector<Mesh> ms(9);
        std::vector<nlfem_mesh> mm;
        std::vector<nlfem_params> pp;
        for (int i = 0; i < 9; ++i) {
            const int n = 7 + (i % 3);
            const double d = (2.0 + 0.5 * (i % 2)) / n;
            kuhn(n, d, ms[(size_t)i]);
            mm.push_back(ms[(size_t)i].m);
            pp.push_back(params(d, 8 + 8 * (i % 2)));
        }
        nlfem_batch* b = nullptr;
        check(nlfem_batch_create(ctx, 9, mm.data(), pp.data(), &b) == NLFEM_OK, "batch_create");
        if (b) {
            check(nlfem_batch_assemble(b, nullptr, nullptr) == NLFEM_OK, "batch_assemble 1");
            check(nlfem_batch_assemble(b, nullptr, nullptr) == NLFEM_OK, "batch_assemble 2");
            int32_t blk = 0, grid = 0;
            double tms = 0.0, lms = 0.0;
            check(nlfem_batch_tuning(b, &blk, &grid, &tms, &lms) == NLFEM_OK, "batch_tuning");
            std::printf("batch: block %d grid %d\n", blk, grid);
            check(nlfem_batch_destroy(b) == NLFEM_OK, "batch_destroy");
        }
        ms[4].tets[3] = -1;
        mm[4] = ms[4].m;
        nlfem_batch* bad = nullptr;
        check(nlfem_batch_create(ctx, 9, mm.data(), pp.data(), &bad) == NLFEM_E_MESH, "failing batch reported");
        check(bad == nullptr, "no batch after a failure");
    }
    check(nlfem_trim(ctx) == NLFEM_OK, "trim");
    check(nlfem_destroy(ctx) == NLFEM_OK, "destroy");
    // the server: two slots, six requests
    {
        nlfem_server* sv = nullptr;
        check(nlfem_server_create(0, 2, (size_t)2 << 30, &sv) == NLFEM_OK, "server_create");
        if (sv) {
            std::vector<Mesh> ms(6);
            std::vector<uint64_t> tk(6, 0);
            for (int i = 0; i < 6; ++i) {
                const int n = 7 + (i % 3);
                const double d = 2.0 / n;
                kuhn(n, d, ms[(size_t)i]);
                nlfem_params p = params(d, 8);
                p.precision = i % 2 ? NLFEM_FP32_LOCAL : NLFEM_FP64;
                check(nlfem_server_submit(sv, &ms[(size_t)i].m, &p, ms[(size_t)i].f.data(), ms[(size_t)i].g.data(),
                                          nullptr, &tk[(size_t)i]) == NLFEM_OK,
                      "server_submit");
            }
            for (int i = 0; i < 6; ++i) {
                nlfem_request_info info{};
                check(nlfem_server_wait(sv, tk[(size_t)i], 120.0, &info) == NLFEM_OK, "server_wait");
                check(info.state == 2, "request done");
                std::vector<double> x((size_t)(info.n_free ? info.n_free : 1));
                std::vector<int32_t> f2v(x.size());
                check(nlfem_server_take(sv, tk[(size_t)i], x.data(), f2v.data()) == NLFEM_OK, "server_take");
            }
            nlfem_server_counters c{};
            check(nlfem_server_stats(sv, &c) == NLFEM_OK, "server_stats");
            std::printf("server: done %lld failed %lld max running %d\n", (long long)c.done, (long long)c.failed,
                        c.max_running);
            check(nlfem_server_destroy(sv) == NLFEM_OK, "server_destroy");
        }
    }
    if (failures) return 1;
    std::printf("ok\n");
    return 0;
}
