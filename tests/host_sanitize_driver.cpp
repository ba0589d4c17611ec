// Host-side setup code of the library (reference element, connectivity,
// blocked trace map, table checks, SARK coefficients) driven on meshes read
// from files, for a build with the address and undefined-behaviour
// sanitizers (tests/test_host_tables.py compiles and runs it).
//
// File layout (little endian): int32 dim, int32 N, int64 nv, int64 K,
// double vx[nv][dim], int32 etov[K][dim+1], double period[dim],
// int8 has_tag, int8 tag[K][dim+1] (when has_tag).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <string>
#include <vector>

#include "../paper_2607_00199_amd/csrc/host_ref.hpp"

namespace {
template <typename T>
bool rd(std::ifstream &f, T *p, size_t n) {
    f.read(reinterpret_cast<char *>(p), std::streamsize(n * sizeof(T)));
    return bool(f);
}

int run_mesh(const char *path) {
    std::ifstream f(path, std::ios::binary);
    int32_t dim = 0, N = 0;
    int64_t nv = 0, K = 0;
    if (!rd(f, &dim, 1) || !rd(f, &N, 1) || !rd(f, &nv, 1) || !rd(f, &K, 1)) return 2;
    std::vector<double> vx(static_cast<size_t>(nv) * dim), period(static_cast<size_t>(dim));
    std::vector<int32_t> etov(size_t(K) * (dim + 1));
    int8_t has_tag = 0;
    if (!rd(f, vx.data(), vx.size()) || !rd(f, etov.data(), etov.size()) || !rd(f, period.data(), period.size()) ||
        !rd(f, &has_tag, 1))
        return 2;
    std::vector<int8_t> tag;
    if (has_tag) {
        tag.resize(size_t(K) * (dim + 1));
        if (!rd(f, tag.data(), tag.size())) return 2;
    }
    const gbh::RefElement ref = gbh::build_ref_element(dim, N, 0);
    std::string err;
    const gbh::Connectivity conn = gbh::build_connectivity(ref, nv, vx.data(), K, etov.data(), period.data(),
                                                           has_tag ? tag.data() : nullptr, err);
    if (!err.empty()) {
        std::printf("%s: connectivity: %s\n", path, err.c_str());
        return 1;
    }
    const std::vector<int32_t> blk = gbh::blocked_trace_map(ref, K, conn);
    const std::string bad = gbh::check_mesh_tables(ref, nv, K, etov.data(), conn, blk);
    if (!bad.empty()) {
        std::printf("%s: tables: %s\n", path, bad.c_str());
        return 1;
    }
    // a batched class of three copies of this mesh, with the buffer sizes the
    // library allocates, and one with a buffer one group too short
    const int NF = dim == 2 ? 6 : 10, NFT = ref.Nfaces * ref.Nfp, slots = (NFT + 3) / 4 * 4;
    std::vector<gbh::BatchMemberLayout> lay(3);
    std::vector<int32_t> gbeg(3);
    const int64_t groups = (K + 15) / 16;
    for (int i = 0; i < 3; ++i) {
        lay[i].K = K;
        lay[i].nv = nv;
        lay[i].etov_bytes = size_t(K) * (dim + 1) * 4;
        lay[i].vstage_bytes = 5 * size_t(nv) * dim * 8;
        lay[i].wstage_bytes = 4 * size_t(nv) * dim * 8;
        lay[i].vmap_bytes = size_t(groups) * slots * 16 * 4;
        lay[i].state_bytes = size_t(groups) * 16 * NF * ref.Np * 8;
        gbeg[i] = int32_t(i * groups);
    }
    if (!gbh::check_batch_class(dim, ref.Np, NF, NFT, 8, lay, gbeg, 3 * groups, 1024, 1000, 65536).empty()) {
        std::printf("%s: a valid batch class was refused\n", path);
        return 1;
    }
    lay[1].state_bytes -= size_t(16) * NF * ref.Np * 8;
    if (gbh::check_batch_class(dim, ref.Np, NF, NFT, 8, lay, gbeg, 3 * groups, 1024, 1000, 65536).empty()) {
        std::printf("%s: a short state buffer was not caught\n", path);
        return 1;
    }
    std::printf("%s: ok (K=%lld, N=%d)\n", path, (long long)K, N);
    return 0;
}
}  // namespace

int main(int argc, char **argv) {
    // every reference element the library builds, and the SARK coefficients
    for (int dim = 2; dim <= 3; ++dim)
        for (int N = 1; N <= (dim == 2 ? 6 : 4); ++N) {
            const gbh::RefElement r = gbh::build_ref_element(dim, N, 0);
            if (r.Np <= 0 || int(r.fmask.size()) != r.Nfaces * r.Nfp) {
                std::printf("reference element %d/%d is inconsistent\n", dim, N);
                return 1;
            }
        }
    for (double g : {0.0, -1e-8, -1e-3, -0.5, -2.0, -20.0, -1e3}) {
        const gbh::SarkCoef c = gbh::sark_coefficients(g);
        double sum = 0.0;
        for (double b : c.b) sum += b;
        if (!(c.E[4] >= 0.0) || !std::isfinite(sum)) {
            std::printf("SARK coefficients at gamma = %g are not finite\n", g);
            return 1;
        }
    }
    int rc = 0;
    for (int i = 1; i < argc; ++i) rc |= run_mesh(argv[i]);
    return rc;
}
