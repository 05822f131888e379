// Forward model kernels (paper Sec. 3.2-3.3) and the synthetic-spot simulator
// (Sec. 3.3.1).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"

namespace laue {

constexpr int kMaxPlanes = 1024;
constexpr int kEnumChunk = 16;   // grains per enumerate work item
constexpr int kEmitList = 2048;  // LDS list of the write pass (>= the bits of 64 mask words)
// a write-pass list entry: grain in chunk << 10 | plane, in 16 bits
static_assert(kMaxPlanes <= 1024 && kEnumChunk <= 64, "write-pass list entries are 16 bits");

// ---------------------------------------------------------------- grains

__global__ void k_set_i64_fwd(int64_t *p, int64_t v) { *p = v; }

__global__ void k_grain_prep(const double *__restrict__ q, const double *__restrict__ x, int n,
                             GrainF *__restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = grain_f32(q + 4 * i, x + 3 * i);
}

int prep_grains(const laue_grains *g, GrainF *dst, hipStream_t s) {
    if (g->n == 0) return LAUE_OK;
    k_grain_prep<<<(g->n + 255) / 256, 256, 0, s>>>(g->q, g->x, g->n, dst);
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}

// ---------------------------------------------------------------- enumerate

// One wave per workgroup, looping over (grain n, rotation t) items.  Phase 1
// marks, per detector, every plane whose spot is in band and on the detector
// (the literal set): first the wavelength of every plane (u_x of Gamma_t R w,
// lambda = 2 d u_x, the arithmetic of spot_geometry), the planes in band
// gathered into an LDS list by ballot; then the full geometry of the listed
// planes only (most planes are out of band), so a wave computes detector
// intersections for in-band planes without idle lanes.  Phase 2 walks the same
// list, applies the harmonic merge (drop a plane if a lower-order parallel
// plane is visible on the same detector) and either counts (pass 0) or writes
// (pass 1) the kept spots in (t, d, n, m) order.
__global__ __launch_bounds__(64) void k_enumerate(
    const GeomF *__restrict__ Gp, const float *__restrict__ W, const float *__restrict__ Dsp,
    const int *__restrict__ prev, int M, const GrainF *__restrict__ grains, int N, int T, int merge,
    int pass, int *__restrict__ counts, const int64_t *__restrict__ offs, int *__restrict__ o_plane,
    int *__restrict__ o_grain, int *__restrict__ o_block, float *__restrict__ o_s1,
    float *__restrict__ o_s2, float *__restrict__ o_vn, float *__restrict__ o_v1,
    float *__restrict__ o_v2, float *__restrict__ o_lam, uint8_t *__restrict__ o_flags,
    unsigned *__restrict__ kmask, int W32, int64_t n_total) {
    const GeomF &G = *Gp;
    const int lane = threadIdx.x;
    // kmask (may be NULL): per item (t, n) and detector, W32 words of kept-plane
    // bits (bit m of word m / 32), written by the count pass for
    // k_enumerate_emit.
    __shared__ unsigned kbits[2 * (kMaxPlanes / 32)];
    // visibility per (detector, plane): dynamic LDS of n_det x M bytes
    extern __shared__ uint8_t vis_lds[];
    __shared__ short inb[kMaxPlanes];
    // the harmonic parents, read by chains of dependent lookups: from LDS
    __shared__ short pv[kMaxPlanes];
    for (int m = lane; m < M; m += 64) pv[m] = static_cast<short>(prev[m] >= 0 && prev[m] < M ? prev[m] : -1);
    __syncthreads();
    const int D = G.n_det;
    // work items: (rotation t, kEnumChunk consecutive grains), so that the
    // outputs of neighbouring grains (adjacent in every (block, grain, plane)
    // ordered array, runs of a few entries each) are written by one wave and
    // reach memory as whole cache lines
    const int64_t n_chunks = (static_cast<int64_t>(N) + kEnumChunk - 1) / kEnumChunk;
    const int64_t n_work = n_chunks * T;
    for (int64_t wi = blockIdx.x; wi < n_work; wi += gridDim.x) {
        const int t = static_cast<int>(wi / n_chunks);
        const int n_lo = static_cast<int>((wi % n_chunks) * kEnumChunk);
        const int n_hi = std::min(N, n_lo + kEnumChunk);
        const float c = G.cs[t][0], s = G.cs[t][1];
        for (int n = n_lo; n < n_hi; ++n) {
            const int64_t item = static_cast<int64_t>(t) * N + n;
            const GrainF gr = grains[n];
            if (!pass && kmask)
                for (int w = lane; w < D * W32; w += 64) kbits[w] = 0u;
            int K = 0;
            for (int m0 = 0; m0 < M; m0 += 64) {
                const int m = m0 + lane;
                bool ib = false;
                if (m < M) {
                    float ux, uy, uz;
                    lab_normal(gr.R, c, s, W[3 * m], W[3 * m + 1], W[3 * m + 2], ux, uy, uz);
                    const float lam = 2.0f * Dsp[m] * ux;
                    ib = (lam >= G.lam_min) && (lam <= G.lam_max);
                    for (int d = 0; d < D; ++d) vis_lds[d * M + m] = 0;
                }
                const unsigned long long bal = __ballot(ib);
                if (ib) inb[K + __popcll(bal & ((1ull << lane) - 1ull))] = static_cast<short>(m);
                K += __popcll(bal);
            }
            __syncthreads();
            for (int k = lane; k < K; k += 64) {
                const int m = inb[k];
                const float wx = W[3 * m], wy = W[3 * m + 1], wz = W[3 * m + 2];
                for (int d = 0; d < D; ++d) {
                    const SpotGeo o = spot_geometry(G, G.det[d], gr.R, gr.x, c, s, wx, wy, wz, Dsp[m]);
                    vis_lds[d * M + m] = (o.inband && o.on) ? 1 : 0;
                }
            }
            __syncthreads();
            for (int d = 0; d < D; ++d) {
                const int slot = (t * D + d) * N + n;
                int64_t base = pass ? offs[slot] : 0;
                int running = 0;
                // visible planes are in band: walk the in-band list (ascending m)
                for (int k0 = 0; k0 < K; k0 += 64) {
                    const int m = k0 + lane < K ? inb[k0 + lane] : 0;
                    bool keep = (k0 + lane < K) && vis_lds[d * M + m];
                    if (merge && keep) {
                        int a = pv[m];
                        for (int hop = 0; hop < 16 && a >= 0; ++hop) {
                            if (vis_lds[d * M + a]) { keep = false; break; }
                            a = pv[a];
                        }
                    }
                    unsigned long long bal = __ballot(keep);
                    if (!pass && kmask && keep) atomicOr(&kbits[d * W32 + (m >> 5)], 1u << (m & 31));
                    const int64_t pos = base + running + __popcll(bal & ((1ull << lane) - 1ull));
                    // (positions outside the output, which only offsets not
                    // made by this set's count could give, are not written)
                    if (pass && keep && pos >= 0 && pos < n_total) {
                        SpotGeo o = spot_geometry(G, G.det[d], gr.R, gr.x, c, s, W[3 * m], W[3 * m + 1],
                                                  W[3 * m + 2], Dsp[m]);
                        o_plane[pos] = m;
                        o_grain[pos] = n;
                        o_block[pos] = t * D + d;
                        if (o_s1) {
                            o_s1[pos] = o.s1;
                            o_s2[pos] = o.s2;
                            o_vn[pos] = o.vn;
                            o_v1[pos] = o.v1;
                            o_v2[pos] = o.v2;
                        }
                        if (o_lam) o_lam[pos] = o.lam;
                        if (o_flags) o_flags[pos] = o.flags;
                    }
                    running += __popcll(bal);
                }
                if (!pass && lane == 0) counts[slot] = running;
            }
            if (!pass && kmask) {
                __syncthreads();
                for (int w = lane; w < D * W32; w += 64) kmask[item * D * W32 + w] = kbits[w];
            }
            __syncthreads();        // vis, inb and kbits are reused by the next item
        }
    }
}

constexpr int kEmitPer = 2;
constexpr int kDetFr = 13;   // floats of a detector frame (DetF) in the write pass's LDS table
static_assert(sizeof(DetF) == kDetFr * sizeof(float), "DetF is 13 floats");

// A wave-uniform value kept in scalar registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
// Inclusive prefix sum over the 64 lanes of a wave by DPP moves: shifts
// by 1, 2, 4 and 8 lanes within each row of 16, then the row broadcasts of
// lane 15 (to rows 1 and 3) and lane 31 (to rows 2 and 3).
__device__ __forceinline__ int wave_incl_scan(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return v;
}
__device__ __forceinline__ int64_t uni(int64_t v) {
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(v)));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(v >> 32)));
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

// Output element idx of array a: a + b0 + off, where off (entries from b0)
// is a 32-bit byte offset from a uniform base when NARROW (fewer than 2^30
// entries from b0), else 64-bit.
template <bool NARROW, typename T>
__device__ __forceinline__ void emit_store(T *__restrict__ a, int64_t b0, int64_t off, T v) {
    if constexpr (NARROW) {
        char *base = reinterpret_cast<char *>(a + b0);
        *reinterpret_cast<T *>(base + (static_cast<uint32_t>(off) * static_cast<uint32_t>(sizeof(T)))) = v;
    } else {
        a[b0 + off] = v;
    }
}

template <bool NARROW>
__device__ __forceinline__ void emit_rows(const GeomF &G, const float *__restrict__ W, const float *__restrict__ Dsp,
                                          const float *gsh, int n_lo, int t, float c, float s,
                                          const uint16_t *elist, int cnt, int s1, int d0, int d1, int64_t b0,
                                          int64_t delta, const float *dfr, int M,
                                          int *__restrict__ o_plane, int *__restrict__ o_grain,
                                          int *__restrict__ o_block, float *__restrict__ o_s1,
                                          float *__restrict__ o_s2, float *__restrict__ o_vn,
                                          float *__restrict__ o_v1, float *__restrict__ o_v2,
                                          float *__restrict__ o_lam, uint8_t *__restrict__ o_flags) {
    for (int k0 = 0; k0 < cnt; k0 += 64 * kEmitPer) {
        int e[kEmitPer];
        float wx[kEmitPer], wy[kEmitPer], wz[kEmitPer], ds[kEmitPer];
#pragma unroll
        for (int j = 0; j < kEmitPer; ++j) {
            const int k = k0 + 64 * j + static_cast<int>(threadIdx.x);
            e[j] = k < cnt ? elist[k] : 0;
            const int m = min(e[j] & 1023, M - 1);        // (bits beyond the plane list are never set)
            wx[j] = W[3 * m];
            wy[j] = W[3 * m + 1];
            wz[j] = W[3 * m + 2];
            ds[j] = Dsp[m];
        }
#pragma unroll
        for (int j = 0; j < kEmitPer; ++j) {
            const int k = k0 + 64 * j + static_cast<int>(threadIdx.x);
            if (k >= cnt) break;
            const int nrel = e[j] >> 10, m = e[j] & 1023;
            const bool hi = k >= s1;
            const float *F = dfr + kDetFr * (hi ? d1 : d0);
            DetF Dd;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                Dd.c[r] = F[r];
                Dd.n[r] = F[3 + r];
                Dd.a1[r] = F[6 + r];
                Dd.a2[r] = F[9 + r];
            }
            Dd.half = F[12];
            const SpotGeo o = spot_geometry(G, Dd, gsh + 12 * nrel, gsh + 12 * nrel + 9, c, s, wx[j], wy[j], wz[j],
                                            ds[j]);
            const int64_t off = hi ? delta + k : k;
            emit_store<NARROW>(o_plane, b0, off, m);
            emit_store<NARROW>(o_grain, b0, off, n_lo + nrel);
            emit_store<NARROW>(o_block, b0, off, t * G.n_det + (hi ? d1 : d0));
            if (o_s1) {
                emit_store<NARROW>(o_s1, b0, off, o.s1);
                emit_store<NARROW>(o_s2, b0, off, o.s2);
                emit_store<NARROW>(o_vn, b0, off, o.vn);
                emit_store<NARROW>(o_v1, b0, off, o.v1);
                emit_store<NARROW>(o_v2, b0, off, o.v2);
            }
            if (o_lam) emit_store<NARROW>(o_lam, b0, off, o.lam);
            if (o_flags) emit_store<NARROW>(o_flags, b0, off, o.flags);
        }
    }
}

// Evaluates and writes the cnt listed (grain in chunk << 10 | plane) entries
// of a work item, read after a barrier (the list may be refilled after the
// closing one).  The list holds at most two detector runs: entries [0, s1) of
// detector d0 go to b0, b0 + 1, ..., entries [s1, cnt) of detector d1 to b1,
// b1 + 1, ... (b1 - s1 >= b0: detector d1's outputs follow d0's).  Every lane
// takes kEmitPer entries at a time and gathers their planes before it writes
// anything: on this chip one counter tracks both the loads and the stores of
// a wave, so a gather issued after a store would also wait for that store to
// complete.  The chunk's grains are in LDS (gsh).
__device__ __forceinline__ void emit_list(const GeomF &G, const float *__restrict__ W, const float *__restrict__ Dsp,
                                          int M, int64_t n_total, const float *gsh, const float *dfr, int n_lo,
                                          int t, float c, float s,
                                          const uint16_t *elist, int cnt, int s1, int d0, int d1, int64_t b0,
                                          int64_t b1, int *__restrict__ o_plane, int *__restrict__ o_grain,
                                          int *__restrict__ o_block, float *__restrict__ o_s1,
                                          float *__restrict__ o_s2, float *__restrict__ o_vn,
                                          float *__restrict__ o_v1, float *__restrict__ o_v2,
                                          float *__restrict__ o_lam, uint8_t *__restrict__ o_flags) {
    __syncthreads();
    b0 = uni(b0);
    const bool two = s1 <= cnt;
    const int64_t delta = uni(two ? b1 - s1 - b0 : int64_t{0});
    // the list's output ranges lie in [0, n_total) for offsets made by this
    // set's count; a list that would leave it is not written
    const bool inside = b0 >= 0 && b0 + (two ? s1 : cnt) <= n_total &&
                        (!two || (b1 >= 0 && b1 + (cnt - s1) <= n_total));
    if (!inside) {
    } else if (delta >= 0 && delta + cnt < (int64_t{1} << 30))
        emit_rows<true>(G, W, Dsp, gsh, n_lo, t, c, s, elist, cnt, s1, d0, d1, b0, delta, dfr, M, o_plane, o_grain,
                        o_block, o_s1, o_s2, o_vn, o_v1, o_v2, o_lam, o_flags);
    else
        emit_rows<false>(G, W, Dsp, gsh, n_lo, t, c, s, elist, cnt, s1, d0, d1, b0, delta, dfr, M, o_plane, o_grain,
                         o_block, o_s1, o_s2, o_vn, o_v1, o_v2, o_lam, o_flags);
    __syncthreads();
}

// Write pass from the count pass's kept-plane bits (kmask, W32 words per (t,
// n) item and detector; at most two detectors): per work item (rotation t,
// kEnumChunk grains), the chunk's mask words, grains and per-detector output
// offsets (all prefetched into registers while the previous item was
// processed) go to LDS; then detector by detector the kept (grain, plane)
// pairs are listed in LDS in output order (ballot compaction), and the list
// of both detectors is evaluated and written by every lane: for one detector
// the chunk's outputs are one contiguous range (offsets in (t, d, n) order),
// written in coalesced runs.
constexpr int kEmitPre = 6;   // mask words per lane prefetched (the rest, if any, load in place)
__global__ __launch_bounds__(64) void k_enumerate_emit(
    const GeomF *__restrict__ Gp, const float *__restrict__ W, const float *__restrict__ Dsp, int M,
    const GrainF *__restrict__ grains, int N, int T, const int64_t *__restrict__ offs, int *__restrict__ o_plane,
    int *__restrict__ o_grain, int *__restrict__ o_block, float *__restrict__ o_s1, float *__restrict__ o_s2,
    float *__restrict__ o_vn, float *__restrict__ o_v1, float *__restrict__ o_v2, float *__restrict__ o_lam,
    uint8_t *__restrict__ o_flags, const unsigned *__restrict__ kmask, int W32, int64_t n_total) {
    const GeomF &G = *Gp;
    const int lane = threadIdx.x;
    const int D = G.n_det;
    extern __shared__ unsigned mw[];
    __shared__ uint16_t elist[kEmitList];
    __shared__ float gsh[kEnumChunk * 12];
    __shared__ int64_t bsh[2];
    __shared__ float dfr[2 * kDetFr];      // the (at most two) detector frames
    if (lane < D * kDetFr) dfr[lane] = G.det[lane / kDetFr].c[lane % kDetFr];
    const float *gflat = reinterpret_cast<const float *>(grains);
    const int64_t n_chunks = (static_cast<int64_t>(N) + kEnumChunk - 1) / kEnumChunk;
    const int64_t n_work = n_chunks * T;
    unsigned pm[kEmitPre];
    float pg[3];
    int64_t pb = 0;
    auto prefetch = [&](int64_t wi) {
        const int t = static_cast<int>(wi / n_chunks);
        const int n_lo = static_cast<int>((wi % n_chunks) * kEnumChunk);
        const int ng = std::min(N, n_lo + kEnumChunk) - n_lo;
        const int n_words = ng * D * W32;
        const unsigned *src = kmask + (static_cast<int64_t>(t) * N + n_lo) * D * W32;
#pragma unroll
        for (int j = 0; j < kEmitPre; ++j) {
            const int k = lane + 64 * j;
            pm[j] = k < n_words ? src[k] : 0u;
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int k = lane + 64 * j;
            pg[j] = k < 12 * ng ? gflat[static_cast<int64_t>(n_lo) * 12 + k] : 0.0f;
        }
        pb = lane < D ? offs[(static_cast<int64_t>(t) * D + lane) * N + n_lo] : 0;
    };
    if (static_cast<int64_t>(blockIdx.x) < n_work) prefetch(blockIdx.x);
    for (int64_t wi = blockIdx.x; wi < n_work; wi += gridDim.x) {
        const int t = static_cast<int>(wi / n_chunks);
        const int n_lo = static_cast<int>((wi % n_chunks) * kEnumChunk);
        const int n_hi = std::min(N, n_lo + kEnumChunk);
        const float c = G.cs[t][0], s = G.cs[t][1];
        const int n_words = (n_hi - n_lo) * D * W32;
#pragma unroll
        for (int j = 0; j < kEmitPre; ++j) {
            const int k = lane + 64 * j;
            if (k < n_words) mw[k] = pm[j];
        }
        const unsigned *src = kmask + (static_cast<int64_t>(t) * N + n_lo) * D * W32;
        for (int k = 64 * kEmitPre + lane; k < n_words; k += 64) mw[k] = src[k];
#pragma unroll
        for (int j = 0; j < 3; ++j) gsh[lane + 64 * j] = pg[j];
        if (lane < D) bsh[lane] = pb;
        __syncthreads();
        if (wi + gridDim.x < n_work) prefetch(wi + gridDim.x);
        // the list: run of detector d0 from b0, then (from entry s1) detector d1 from b1
        int cnt = 0, s1 = kEmitList + 1, d0 = 0, d1 = 0;
        int64_t b0 = 0, b1 = 0;
        for (int d = 0; d < D; ++d) {
            if (cnt == 0) {
                d0 = d;
                b0 = uni(bsh[d]);
                s1 = kEmitList + 1;
            } else {
                d1 = d;
                b1 = uni(bsh[d]);
                s1 = cnt;
            }
            // the chunk's mask words of detector d in (grain, word) order, 64
            // at a time: each lane lists the set bits of its word at its
            // scanned position, so the list stays in (grain, plane) order
            const int nw = (n_hi - n_lo) * W32;
            for (int r0 = 0; r0 < nw; r0 += 64) {
                const int idx = r0 + lane;
                unsigned word = 0u;
                int nrel = 0, w = 0;
                if (idx < nw) {
                    nrel = idx / W32;
                    w = idx - nrel * W32;
                    word = mw[(nrel * D + d) * W32 + w];
                }
                const int pc = __popc(word);
                const int incl = wave_incl_scan(pc);
                const int total = __builtin_amdgcn_readlane(incl, 63);
                if (cnt + total > kEmitList) {        // no room for this round: write the list out
                    emit_list(G, W, Dsp, M, n_total, gsh, dfr, n_lo, t, c, s, elist, cnt, s1, d0, d1, b0, b1, o_plane, o_grain,
                              o_block, o_s1, o_s2, o_vn, o_v1, o_v2, o_lam, o_flags);
                    // detector d goes on in a new list
                    const int64_t next = s1 <= cnt ? b1 + (cnt - s1) : b0 + cnt;
                    cnt = 0;
                    d0 = d;
                    b0 = next;
                    s1 = kEmitList + 1;
                }
                int q = cnt + incl - pc;
                for (unsigned wb = word; wb; wb &= wb - 1u)
                    elist[q++] = static_cast<uint16_t>((nrel << 10) | (w * 32 + __ffs(wb) - 1));
                cnt += total;
            }
        }
        if (cnt > 0)
            emit_list(G, W, Dsp, M, n_total, gsh, dfr, n_lo, t, c, s, elist, cnt, s1, d0, d1, b0, b1, o_plane, o_grain, o_block,
                      o_s1, o_s2, o_vn, o_v1, o_v2, o_lam, o_flags);
        __syncthreads();        // mw, gsh and bsh are reused by the next work item
    }
}

// Workgroups of k_enumerate: all resident at once (32 one-wave workgroups per
// CU, 4 KB of static and n_det x M bytes of dynamic LDS each), at most one per
// item; enum_lds is the dynamic part.
unsigned enum_grid(int N, int T) {
    const int64_t chunks = (static_cast<int64_t>(N) + kEnumChunk - 1) / kEnumChunk;
    return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(chunks * T, 256 * 32)));
}
size_t enum_lds(int n_det, int M) { return static_cast<size_t>(n_det) * M; }
// Workgroups of k_enumerate_emit: all resident at once (20 one-wave
// workgroups per CU, bound by its vector registers), at most one per item.
unsigned emit_grid(int N, int T) {
    const int64_t chunks = (static_cast<int64_t>(N) + kEnumChunk - 1) / kEnumChunk;
    return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(chunks * T, 256 * 20)));
}

// Exclusive scan of L int counts into out[0 .. L] (out[L] = total), over
// the whole GPU in three launches and no memory beyond out: chunks of
// kScanChunk counts (kScanPerThread per thread of a 256-thread workgroup).
// (1) each chunk's sum goes to out[chunk start]; (2) one workgroup scans those
// sums in place, which leaves at each chunk start its exclusive prefix, i.e.
// the chunk's offset, and writes the total to out[L]; (3) each chunk scans its
// counts from that offset.  Fixed order everywhere: the result is the exact
// integer scan.
constexpr int kScanPerThread = 16;
constexpr int kScanChunk = 256 * kScanPerThread;

__device__ __forceinline__ int64_t block_exclusive_scan_256(int64_t v, int64_t *sh, int64_t *total) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int64_t t = tid >= o ? sh[tid - o] : 0;
        __syncthreads();
        sh[tid] += t;
        __syncthreads();
    }
    const int64_t incl = sh[tid];
    if (total) *total = sh[255];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(256) void k_scan_part(const int *__restrict__ in, int64_t *__restrict__ out,
                                                   int64_t L) {
    __shared__ int64_t sh[256];
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * kScanChunk;
    const int64_t i0 = c0 + static_cast<int64_t>(threadIdx.x) * kScanPerThread;
    int64_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k)
        if (i0 + k < L) sum += in[i0 + k];
    int64_t tot = 0;
    block_exclusive_scan_256(sum, sh, &tot);
    if (threadIdx.x == 0) out[c0] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_top(int64_t *__restrict__ out, int64_t L, int64_t n_chunks) {
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x;
    const int64_t per = (n_chunks + 1023) / 1024;
    const int64_t b0 = std::min<int64_t>(n_chunks, tid * per), b1 = std::min<int64_t>(n_chunks, b0 + per);
    int64_t sum = 0;
    for (int64_t b = b0; b < b1; ++b) sum += out[b * kScanChunk];
    part[tid] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int64_t t = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += t;
        __syncthreads();
    }
    int64_t run = part[tid] - sum;
    for (int64_t b = b0; b < b1; ++b) {
        const int64_t v = out[b * kScanChunk];
        out[b * kScanChunk] = run;
        run += v;
    }
    if (tid == 1023) out[L] = part[1023];
}

__global__ __launch_bounds__(256) void k_scan_fill(const int *__restrict__ in, int64_t *__restrict__ out,
                                                   int64_t L) {
    __shared__ int64_t sh[256];
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * kScanChunk;
    const int64_t base = out[c0];
    __syncthreads();            // every thread has read the offset before thread 0 rewrites out[c0]
    const int64_t i0 = c0 + static_cast<int64_t>(threadIdx.x) * kScanPerThread;
    int v[kScanPerThread];
    int64_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        v[k] = i0 + k < L ? in[i0 + k] : 0;
        sum += v[k];
    }
    int64_t run = base + block_exclusive_scan_256(sum, sh, nullptr);
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k)
        if (i0 + k < L) {
            out[i0 + k] = run;
            run += v[k];
        }
}

// blk[b] = out[min(L, b * stride)] for b <= n_blocks
__global__ void k_scan_blocks(const int64_t *__restrict__ out, int64_t L, int64_t *__restrict__ blk, int n_blocks,
                              int64_t stride) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b <= n_blocks) blk[b] = out[std::min<int64_t>(L, b * stride)];
}

int launch_scan(const int *in, int64_t *out, int64_t L, hipStream_t s) {
    if (L <= 0) {
        k_set_i64_fwd<<<1, 1, 0, s>>>(out, 0);
        LAUE_CHECK_HIP(hipGetLastError());
        return LAUE_OK;
    }
    const int64_t nc = (L + kScanChunk - 1) / kScanChunk;
    k_scan_part<<<static_cast<unsigned>(nc), 256, 0, s>>>(in, out, L);
    k_scan_top<<<1, 1024, 0, s>>>(out, L, nc);
    k_scan_fill<<<static_cast<unsigned>(nc), 256, 0, s>>>(in, out, L);
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}

// ---------------------------------------------------------------- eval

__global__ void k_eval(const GeomF *__restrict__ Gp, const float *__restrict__ W,
                       const float *__restrict__ Dsp, const GrainF *__restrict__ grains,
                       const int *__restrict__ plane, const int *__restrict__ grain,
                       const int *__restrict__ block, int64_t n, int n_planes, int n_grains,
                       float *__restrict__ o_s1,
                       float *__restrict__ o_s2, float *__restrict__ o_vn,
                       float *__restrict__ o_v1, float *__restrict__ o_v2,
                       float *__restrict__ o_lam, Col8 *__restrict__ cols) {
    int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const GeomF &G = *Gp;
    int m = plane[j], g = grain[j], b = block[j];
    if (m < 0 || m >= n_planes || g < 0 || g >= n_grains || b < 0 || b >= G.n_rot * G.n_det) {
        // invalid ids: no geometry (NaN) rather than an out-of-bounds read
        const float nan = __builtin_nanf("");
        if (o_s1) { o_s1[j] = nan; o_s2[j] = nan; o_vn[j] = nan; o_v1[j] = nan; o_v2[j] = nan; }
        if (o_lam) o_lam[j] = nan;
        if (cols) cols[j] = Col8{nan, nan, nan, nan, nan, nan, nan, 0.0f};
        return;
    }
    int t = b / G.n_det, d = b - t * G.n_det;
    const GrainF &gr = grains[g];
    SpotGeo o = spot_geometry(G, G.det[d], gr.R, gr.x, G.cs[t][0], G.cs[t][1], W[3 * m],
                              W[3 * m + 1], W[3 * m + 2], Dsp[m]);
    if (o_s1) {
        o_s1[j] = o.s1;
        o_s2[j] = o.s2;
        o_vn[j] = o.vn;
        o_v1[j] = o.v1;
        o_v2[j] = o.v2;
    }
    if (o_lam) o_lam[j] = o.lam;
    if (cols) {
        Col8 c;
        c.s1 = o.s1;
        c.s2 = o.s2;
        c.v1 = o.v1;
        c.v2 = o.v2;
        c.vv = fmaf(o.v2, o.v2, fmaf(o.v1, o.v1, o.vn * o.vn));
        c.vv2 = c.vv * c.vv;
        c.vn = o.vn;
        c.pad = 0.0f;
        cols[j] = c;
    }
}

__global__ void k_pack_cols(const float *__restrict__ s1, const float *__restrict__ s2,
                            const float *__restrict__ vn, const float *__restrict__ v1,
                            const float *__restrict__ v2, int64_t n, Col8 *__restrict__ cols) {
    int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= n) return;
    Col8 c;
    c.s1 = s1[j];
    c.s2 = s2[j];
    c.v1 = v1[j];
    c.v2 = v2[j];
    c.vv = fmaf(v2[j], v2[j], fmaf(v1[j], v1[j], vn[j] * vn[j]));
    c.vv2 = c.vv * c.vv;
    c.vn = vn[j];
    c.pad = 0.0f;
    cols[j] = c;
}

int launch_eval(const GeomF *dG, const laue_planes *pl, const GrainF *dgr, int n_grains,
                const int *plane, const int *grain, const int *block, int64_t n, float *s1,
                float *s2, float *vn, float *v1, float *v2, float *lam, Col8 *cols, hipStream_t s) {
    if (n == 0) return LAUE_OK;
    int64_t nb = (n + 255) / 256;
    k_eval<<<static_cast<unsigned>(nb), 256, 0, s>>>(dG, pl->w, pl->d, dgr, plane, grain, block,
                                                     n, pl->n, n_grains, s1, s2, vn, v1, v2, lam,
                                                     cols);
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}

int launch_pack(const laue_model_spots *m, Col8 *cols, hipStream_t s) {
    if (m->n == 0) return LAUE_OK;
    int64_t nb = (m->n + 255) / 256;
    k_pack_cols<<<static_cast<unsigned>(nb), 256, 0, s>>>(m->s1, m->s2, m->vn, m->v1, m->v2, m->n,
                                                          cols);
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}

int validate_planes(const laue_planes *p) {
    LAUE_REQUIRE(p != nullptr && p->w && p->d && p->harmonic_prev, LAUE_EINVAL,
                 "planes or one of its arrays is NULL");
    LAUE_REQUIRE(p->n >= 1 && p->n <= kMaxPlanes, LAUE_EINVAL, "n_planes must be in 1..1024");
    return LAUE_OK;
}

int validate_grains(const laue_grains *g) {
    LAUE_REQUIRE(g != nullptr && g->n >= 0, LAUE_EINVAL, "grains is NULL or n < 0");
    LAUE_REQUIRE(g->n == 0 || (g->q && g->x), LAUE_EINVAL, "grain arrays are NULL");
    return LAUE_OK;
}

size_t carve_enum(Carver &cv, EnumWs &w, const laue_geometry *g, int n_grains, int n_planes) {
    int64_t L = static_cast<int64_t>(g->n_rot) * g->n_det * std::max(n_grains, 1);
    w.geom = cv.take<GeomF>(1);
    w.grains = cv.take<GrainF>(std::max(n_grains, 1));
    w.counts = cv.take<int>(L);
    w.offs = cv.take<int64_t>(L + 1);
    w.blk = cv.take<int64_t>(g->n_rot * g->n_det + 1);
    // kept-plane bits of the count pass (not when a plane list is larger
    // than the kernel's limit or the geometry has more than two detectors)
    w.w32 = (std::min(std::max(n_planes, 1), kMaxPlanes) + 31) / 32;
    w.kmask = g->n_det <= 2 ? cv.take<unsigned>(L * w.w32) : nullptr;
    w.mask_ready = false;
    return cv.size();
}

// Count pass, scan and block offsets of the (merged) visible set.  Leaves
// host_blk filled; returns the total in *total.
int enumerate_count(const laue_geometry *geom, const laue_planes *planes,
                           const laue_grains *grains, int merge, EnumWs &w,
                           std::vector<int64_t> &host_blk, int64_t *total, hipStream_t s) {
    GeomF hg;
    make_geomf(geom, &hg);
    LAUE_CHECK_HIP(hipMemcpyAsync(w.geom, &hg, sizeof(GeomF), hipMemcpyHostToDevice, s));
    int rc = prep_grains(grains, w.grains, s);
    if (rc) return rc;
    const int N = grains->n;
    const int nb = geom->n_rot * geom->n_det;
    host_blk.assign(nb + 1, 0);
    if (N == 0) {
        *total = 0;
        LAUE_CHECK_HIP(hipStreamSynchronize(s));
        return LAUE_OK;
    }
    const int64_t L = static_cast<int64_t>(geom->n_rot) * geom->n_det * N;
    unsigned *mask = w.kmask && planes->n <= 32 * w.w32 ? w.kmask : nullptr;
    k_enumerate<<<enum_grid(N, geom->n_rot), 64, enum_lds(geom->n_det, planes->n), s>>>(w.geom, planes->w, planes->d, planes->harmonic_prev,
                                               planes->n, w.grains, N, geom->n_rot, merge, 0, w.counts, nullptr,
                                               nullptr, nullptr, nullptr, nullptr, nullptr,
                                               nullptr, nullptr, nullptr, nullptr, nullptr, mask, w.w32, 0);
    LAUE_CHECK_HIP(hipGetLastError());
    w.mask_ready = mask != nullptr;
    if ((rc = launch_scan(w.counts, w.offs, L, s))) return rc;
    k_scan_blocks<<<(nb + 1 + 255) / 256, 256, 0, s>>>(w.offs, L, w.blk, nb, N);
    LAUE_CHECK_HIP(hipGetLastError());
    LAUE_CHECK_HIP(hipMemcpyAsync(host_blk.data(), w.blk, (nb + 1) * sizeof(int64_t),
                                  hipMemcpyDeviceToHost, s));
    LAUE_CHECK_HIP(hipStreamSynchronize(s));
    *total = host_blk[nb];
    return LAUE_OK;
}

// Write pass after enumerate_count on the same workspace: from the count
// pass's kept-plane bits when it wrote them, else recomputing every plane.
int launch_emit(const laue_geometry *geom, const laue_planes *planes, EnumWs &w, int N, int merge, int64_t n_total,
                int *plane, int *grain, int *block, float *s1, float *s2, float *vn, float *v1, float *v2, float *lam,
                uint8_t *flags, hipStream_t s) {
    if (N == 0) return LAUE_OK;
    if (w.mask_ready)
        k_enumerate_emit<<<emit_grid(N, geom->n_rot), 64,
                           static_cast<size_t>(kEnumChunk) * geom->n_det * w.w32 * sizeof(unsigned), s>>>(
            w.geom, planes->w, planes->d, planes->n, w.grains, N, geom->n_rot, w.offs, plane, grain, block, s1, s2,
            vn, v1, v2, lam, flags, w.kmask, w.w32, n_total);
    else
        k_enumerate<<<enum_grid(N, geom->n_rot), 64, enum_lds(geom->n_det, planes->n), s>>>(
            w.geom, planes->w, planes->d, planes->harmonic_prev, planes->n, w.grains, N, geom->n_rot, merge, 1,
            nullptr, w.offs, plane, grain, block, s1, s2, vn, v1, v2, lam, flags, nullptr, w.w32, n_total);
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}

// Write pass of the enumerate (ids only) after enumerate_count on the same workspace.
int launch_enumerate_ids(const laue_geometry *geom, const laue_planes *planes, EnumWs &w, int N,
                         int merge, int64_t n_total, int *plane, int *grain, int *block, hipStream_t s) {
    return launch_emit(geom, planes, w, N, merge, n_total, plane, grain, block, nullptr, nullptr, nullptr, nullptr,
                       nullptr, nullptr, nullptr, s);
}

// ---------------------------------------------------------------- simulate

__device__ __forceinline__ double u01(uint32_t v) { return (static_cast<double>(v) + 0.5) * (1.0 / 4294967296.0); }

// Noisy ray and detector hit of each visible spot (FP64; the simulator is
// not on the hot path).  keep = tau > 0 and inside the detector square.
__global__ void k_sim_noise(const laue_geometry G, const float *__restrict__ W,
                            const double *__restrict__ q, const double *__restrict__ x,
                            const int *__restrict__ plane, const int *__restrict__ grain,
                            const int *__restrict__ block, int64_t n, double sig, uint32_t k0,
                            uint32_t k1, double *__restrict__ o_p1, double *__restrict__ o_p2,
                            uint8_t *__restrict__ keep, uint64_t *__restrict__ key) {
    int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int m = plane[j], g = grain[j], b = block[j];
    int t = b / G.n_det, d = b - t * G.n_det;
    double qw = q[4 * g], qa = q[4 * g + 1], qb = q[4 * g + 2], qc = q[4 * g + 3];
    double qn = sqrt(qw * qw + qa * qa + qb * qb + qc * qc);
    qw /= qn; qa /= qn; qb /= qn; qc /= qn;
    double R[9] = {1 - 2 * (qb * qb + qc * qc), 2 * (qa * qb - qw * qc), 2 * (qa * qc + qw * qb),
                   2 * (qa * qb + qw * qc), 1 - 2 * (qa * qa + qc * qc), 2 * (qb * qc - qw * qa),
                   2 * (qa * qc - qw * qb), 2 * (qb * qc + qw * qa), 1 - 2 * (qa * qa + qb * qb)};
    double wx = W[3 * m], wy = W[3 * m + 1], wz = W[3 * m + 2];
    double vx = R[0] * wx + R[1] * wy + R[2] * wz;
    double vy = R[3] * wx + R[4] * wy + R[5] * wz;
    double vz = R[6] * wx + R[7] * wy + R[8] * wz;
    double om = G.omega0 + G.domega * t, c = cos(om), s = sin(om);
    double ux = c * vx - s * vy, uy = s * vx + c * vy, uz = vz;
    double r[3] = {1 - 2 * ux * ux, -2 * ux * uy, -2 * ux * uz};
    double y[3] = {c * x[3 * g] - s * x[3 * g + 1], s * x[3 * g] + c * x[3 * g + 1], x[3 * g + 2]};
    uint32_t ctr[4] = {static_cast<uint32_t>(g), static_cast<uint32_t>(t),
                       static_cast<uint32_t>(m + 65536 * d), 1u};
    philox(ctr, k0, k1);
    double z[3];
    {
        double rad = sqrt(-2.0 * log(u01(ctr[0]))), ang = 2.0 * M_PI * u01(ctr[1]);
        z[0] = rad * cos(ang);
        z[1] = rad * sin(ang);
        double rad2 = sqrt(-2.0 * log(u01(ctr[2]))), ang2 = 2.0 * M_PI * u01(ctr[3]);
        z[2] = rad2 * cos(ang2);
    }
    double rn[3];
    double nn = 0;
    for (int k = 0; k < 3; ++k) {
        rn[k] = r[k] + sig * z[k];
        nn += rn[k] * rn[k];
    }
    nn = sqrt(nn);
    for (int k = 0; k < 3; ++k) rn[k] /= nn;
    const laue_detector &D = G.det[d];
    double den = 0, num = 0;
    for (int k = 0; k < 3; ++k) {
        den += D.normal[k] * rn[k];
        num += D.normal[k] * (D.center[k] - y[k]);
    }
    double tau = num / den;
    double p1 = 0, p2 = 0;
    for (int k = 0; k < 3; ++k) {
        double rel = y[k] + tau * rn[k] - D.center[k];
        p1 += D.axis1[k] * rel;
        p2 += D.axis2[k] * rel;
    }
    o_p1[j] = p1;
    o_p2[j] = p2;
    keep[j] = (tau > 0 && fmax(fabs(p1), fabs(p2)) < D.half_size) ? 1 : 0;
    uint32_t kc[4] = {static_cast<uint32_t>(g), static_cast<uint32_t>(t),
                      static_cast<uint32_t>(m + 65536 * d), 3u};
    philox(kc, k0, k1);
    key[j] = (static_cast<uint64_t>(kc[0]) << 32) | kc[1];
}

// Kept true spots per block (one workgroup per block, fixed order).
__global__ __launch_bounds__(256) void k_sim_count(const int64_t *__restrict__ sblk,
                                                   const uint8_t *__restrict__ keep,
                                                   int *__restrict__ n_true) {
    int b = blockIdx.x;
    __shared__ int part[256];
    int c = 0;
    for (int64_t j = sblk[b] + threadIdx.x; j < sblk[b + 1]; j += 256) c += keep[j];
    part[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int k = 0; k < 256; ++k) s += part[k];
        n_true[b] = s;
    }
}

// Per block: gather kept true spots (in visible-set order) and outliers, rank
// them by (key, source, index) and scatter to the output at the block offset.
__global__ __launch_bounds__(256) void k_sim_emit(
    const laue_geometry G, const int64_t *__restrict__ sblk, const uint8_t *__restrict__ keep,
    const double *__restrict__ np1, const double *__restrict__ np2, const uint64_t *__restrict__ key,
    const int *__restrict__ s_plane, const int *__restrict__ s_grain, const int64_t *__restrict__ oblk,
    const int *__restrict__ n_out, uint32_t k0, uint32_t k1, uint64_t *__restrict__ tkey,
    int *__restrict__ tsrc, float *__restrict__ tp1, float *__restrict__ tp2,
    int *__restrict__ tgr, int *__restrict__ tpl, float *__restrict__ p1, float *__restrict__ p2,
    int *__restrict__ o_grain, int *__restrict__ o_plane) {
    const int b = blockIdx.x;
    const int t = b / G.n_det, d = b - t * G.n_det;
    const int64_t base = oblk[b];
    __shared__ int part[256];
    // compaction of kept true spots: thread-contiguous chunks, then a prefix
    const int64_t s0 = sblk[b], s1 = sblk[b + 1], ns = s1 - s0;
    const int64_t chunk = (ns + 255) / 256;
    const int64_t c0 = s0 + std::min<int64_t>(ns, threadIdx.x * chunk);
    const int64_t c1 = s0 + std::min<int64_t>(ns, (threadIdx.x + 1) * chunk);
    int cnt = 0;
    for (int64_t j = c0; j < c1; ++j) cnt += keep[j];
    part[threadIdx.x] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int k = 0; k < 256; ++k) {
            int v = part[k];
            part[k] = run;
            run += v;
        }
    }
    __syncthreads();
    int pos = part[threadIdx.x];
    for (int64_t j = c0; j < c1; ++j) {
        if (!keep[j]) continue;
        int64_t o = base + pos++;
        tkey[o] = key[j];
        tsrc[o] = pos - 1;  // index among kept true spots
        tp1[o] = static_cast<float>(np1[j]);
        tp2[o] = static_cast<float>(np2[j]);
        tgr[o] = s_grain[j];
        tpl[o] = s_plane[j];
    }
    __syncthreads();
    __shared__ int ntrue_s;
    if (threadIdx.x == 255) ntrue_s = part[255] + cnt;
    __syncthreads();
    const int nt = ntrue_s;
    const int no = n_out[b];
    const double side = 2.0 * G.det[d].half_size;
    for (int k = threadIdx.x; k < no; k += 256) {
        uint32_t c[4] = {static_cast<uint32_t>(k), static_cast<uint32_t>(t),
                         static_cast<uint32_t>(65536 * d), 2u};
        philox(c, k0, k1);
        uint32_t kc[4] = {static_cast<uint32_t>(k), static_cast<uint32_t>(t),
                          static_cast<uint32_t>(65536 * d), 4u};
        philox(kc, k0, k1);
        int64_t o = base + nt + k;
        tkey[o] = (static_cast<uint64_t>(kc[0]) << 32) | kc[1];
        tsrc[o] = (1 << 30) + k;
        tp1[o] = static_cast<float>((u01(c[0]) - 0.5) * side);
        tp2[o] = static_cast<float>((u01(c[1]) - 0.5) * side);
        tgr[o] = -1;
        tpl[o] = -1;
    }
    __syncthreads();
    const int tot = nt + no;
    for (int a = threadIdx.x; a < tot; a += 256) {
        const uint64_t ka = tkey[base + a];
        const int sa = tsrc[base + a];
        int rank = 0;
        for (int c = 0; c < tot; ++c) {
            uint64_t kb = tkey[base + c];
            int sb = tsrc[base + c];
            rank += (kb < ka) || (kb == ka && sb < sa);
        }
        int64_t o = base + rank;
        p1[o] = tp1[base + a];
        p2[o] = tp2[base + a];
        o_grain[o] = tgr[base + a];
        o_plane[o] = tpl[base + a];
    }
}

}  // namespace laue

using namespace laue;

extern "C" size_t laue_forward_workspace_size(const laue_geometry *geom, int32_t n_planes,
                                              int32_t n_grains) {
    if (!geom || validate_geometry(geom) != LAUE_OK || n_grains < 0 || n_planes < 0) return 0;
    Carver cv(nullptr);
    EnumWs w;
    return carve_enum(cv, w, geom, n_grains, n_planes);
}

namespace {
// What a count of laue_forward_enumerate left in its workspace: the call's
// sizes, geometry, argument pointers and results, so that
// laue_forward_enumerate_counted can check that it writes the set counted for
// the same arguments.  A few workspaces at a time (most recent first).
struct CountRecord {
    const void *ws = nullptr;
    GeomF geom;
    const float *pw = nullptr, *pd = nullptr;
    const int32_t *pprev = nullptr;
    int32_t n_planes = 0;
    const double *q = nullptr, *x = nullptr;
    int64_t n_grains = 0;
    int merge = 0;
    bool mask_ready = false;
    int64_t total = 0;
    std::vector<int64_t> blk;
};
constexpr size_t kCountRecords = 8;
std::mutex g_count_mu;
std::vector<CountRecord> g_counts;

void remember_count(const void *ws, const laue_geometry *geom, const laue_planes *planes, const laue_grains *grains,
                    int merge, const EnumWs &w, int64_t total, const std::vector<int64_t> &blk) {
    CountRecord r;
    r.ws = ws;
    make_geomf(geom, &r.geom);
    r.pw = planes->w;
    r.pd = planes->d;
    r.pprev = planes->harmonic_prev;
    r.n_planes = planes->n;
    r.q = grains->q;
    r.x = grains->x;
    r.n_grains = grains->n;
    r.merge = merge;
    r.mask_ready = w.mask_ready;
    r.total = total;
    r.blk = blk;
    std::lock_guard<std::mutex> lk(g_count_mu);
    g_counts.erase(std::remove_if(g_counts.begin(), g_counts.end(), [&](const CountRecord &c) { return c.ws == ws; }),
                   g_counts.end());
    g_counts.insert(g_counts.begin(), std::move(r));
    if (g_counts.size() > kCountRecords) g_counts.pop_back();
}
}  // namespace

extern "C" int laue_forward_enumerate(const laue_geometry *geom, const laue_planes *planes,
                                      const laue_grains *grains, int merge_harmonics,
                                      laue_model_spots *out, int64_t *n_out, void *ws,
                                      size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_geometry(geom)) || (rc = validate_planes(planes)) ||
        (rc = validate_grains(grains)))
        return rc;
    LAUE_REQUIRE(out && n_out && out->block_off, LAUE_EINVAL, "output or n_out is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    EnumWs w;
    size_t need = carve_enum(cv, w, geom, grains->n, planes->n);
    if ((rc = check_ws(ws, ws_bytes, need))) return rc;
    std::vector<int64_t> hb;
    int64_t total = 0;
    if ((rc = enumerate_count(geom, planes, grains, merge_harmonics ? 1 : 0, w, hb, &total, s)))
        return rc;
    remember_count(ws, geom, planes, grains, merge_harmonics ? 1 : 0, w, total, hb);
    *n_out = total;
    std::memcpy(out->block_off, hb.data(), hb.size() * sizeof(int64_t));
    if (total > out->n) {
        set_error("model-spot capacity " + std::to_string(out->n) + " < required " +
                  std::to_string(total));
        return LAUE_ECAPACITY;
    }
    if (total > 0) {
        LAUE_REQUIRE(out->plane && out->grain && out->block && out->s1 && out->s2 && out->vn &&
                         out->v1 && out->v2,
                     LAUE_EINVAL, "model-spot arrays are NULL");
        if ((rc = launch_emit(geom, planes, w, grains->n, merge_harmonics ? 1 : 0, total, out->plane, out->grain,
                              out->block, out->s1, out->s2, out->vn, out->v1, out->v2, out->lam, out->flags, s)))
            return rc;
    }
    out->n = total;
    LAUE_CHECK_HIP(hipStreamSynchronize(s));
    return LAUE_OK;
}

extern "C" int laue_forward_enumerate_counted(const laue_geometry *geom, const laue_planes *planes,
                                              const laue_grains *grains, int merge_harmonics,
                                              laue_model_spots *out, int64_t *n_out, void *ws,
                                              size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_geometry(geom)) || (rc = validate_planes(planes)) ||
        (rc = validate_grains(grains)))
        return rc;
    LAUE_REQUIRE(out && n_out && out->block_off, LAUE_EINVAL, "output or n_out is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    EnumWs w;
    size_t need = carve_enum(cv, w, geom, grains->n, planes->n);
    if ((rc = check_ws(ws, ws_bytes, need))) return rc;
    const int merge = merge_harmonics ? 1 : 0;
    GeomF hg;
    make_geomf(geom, &hg);
    CountRecord r;
    bool found = false;
    {
        std::lock_guard<std::mutex> lk(g_count_mu);
        for (const CountRecord &c : g_counts)
            if (c.ws == ws) {
                r = c;
                found = true;
                break;
            }
    }
    LAUE_REQUIRE(found, LAUE_EINVAL, "no laue_forward_enumerate count on this workspace");
    LAUE_REQUIRE(std::memcmp(&r.geom, &hg, sizeof(GeomF)) == 0 && r.pw == planes->w && r.pd == planes->d &&
                     r.pprev == planes->harmonic_prev && r.n_planes == planes->n && r.q == grains->q &&
                     r.x == grains->x && r.n_grains == grains->n && r.merge == merge,
                 LAUE_EINVAL, "arguments differ from those of the count on this workspace");
    if (grains->n > 0) {
        // the count's block offsets must still be in the workspace
        std::vector<int64_t> blk(r.blk.size());
        LAUE_CHECK_HIP(hipMemcpyAsync(blk.data(), w.blk, blk.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        LAUE_CHECK_HIP(hipStreamSynchronize(s));
        LAUE_REQUIRE(blk == r.blk, LAUE_EINVAL, "the workspace no longer holds the count of laue_forward_enumerate");
    }
    *n_out = r.total;
    std::memcpy(out->block_off, r.blk.data(), r.blk.size() * sizeof(int64_t));
    if (r.total > out->n) {
        set_error("model-spot capacity " + std::to_string(out->n) + " < required " + std::to_string(r.total));
        return LAUE_ECAPACITY;
    }
    if (r.total > 0) {
        LAUE_REQUIRE(out->plane && out->grain && out->block && out->s1 && out->s2 && out->vn && out->v1 && out->v2,
                     LAUE_EINVAL, "model-spot arrays are NULL");
        w.mask_ready = r.mask_ready;
        if ((rc = launch_emit(geom, planes, w, grains->n, merge, r.total, out->plane, out->grain, out->block, out->s1,
                              out->s2, out->vn, out->v1, out->v2, out->lam, out->flags, s)))
            return rc;
    }
    out->n = r.total;
    LAUE_CHECK_HIP(hipStreamSynchronize(s));
    return LAUE_OK;
}

extern "C" int laue_forward_eval(const laue_geometry *geom, const laue_planes *planes,
                                 const laue_grains *grains, laue_model_spots *spots, void *ws,
                                 size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_geometry(geom)) || (rc = validate_planes(planes)) ||
        (rc = validate_grains(grains)))
        return rc;
    LAUE_REQUIRE(spots && spots->n >= 0, LAUE_EINVAL, "spots is NULL");
    LAUE_REQUIRE(spots->n == 0 || (spots->plane && spots->grain && spots->block && spots->s1 &&
                                   spots->s2 && spots->vn && spots->v1 && spots->v2),
                 LAUE_EINVAL, "spot arrays are NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    EnumWs w;
    size_t need = carve_enum(cv, w, geom, grains->n, planes->n);
    if ((rc = check_ws(ws, ws_bytes, need))) return rc;
    GeomF hg;
    make_geomf(geom, &hg);
    LAUE_CHECK_HIP(hipMemcpyAsync(w.geom, &hg, sizeof(GeomF), hipMemcpyHostToDevice, s));
    if ((rc = prep_grains(grains, w.grains, s))) return rc;
    rc = launch_eval(w.geom, planes, w.grains, grains->n, spots->plane, spots->grain, spots->block, spots->n,
                     spots->s1, spots->s2, spots->vn, spots->v1, spots->v2, spots->lam, nullptr, s);
    if (rc) return rc;
    // the geometry copy above is from a stack object: wait before returning
    LAUE_CHECK_HIP(hipStreamSynchronize(s));
    return LAUE_OK;
}

struct SimWs {
    EnumWs e;
    int *plane, *grain, *block;
    double *np1, *np2;
    uint8_t *keep;
    uint64_t *key;
    int *n_true, *n_out;
    int64_t *oblk;
    uint64_t *tkey;
    int *tsrc, *tgr, *tpl;
    float *tp1, *tp2;
};

static size_t carve_sim(Carver &cv, SimWs &w, const laue_geometry *g, int n_grains, int64_t n_true_max,
                        int64_t n_obs_max, int n_planes) {
    carve_enum(cv, w.e, g, n_grains, n_planes);
    int64_t S = std::max<int64_t>(n_true_max, 1), O = std::max<int64_t>(n_obs_max, 1);
    int nb = g->n_rot * g->n_det;
    w.plane = cv.take<int>(S);
    w.grain = cv.take<int>(S);
    w.block = cv.take<int>(S);
    w.np1 = cv.take<double>(S);
    w.np2 = cv.take<double>(S);
    w.keep = cv.take<uint8_t>(S);
    w.key = cv.take<uint64_t>(S);
    w.n_true = cv.take<int>(nb);
    w.n_out = cv.take<int>(nb);
    w.oblk = cv.take<int64_t>(nb + 1);
    w.tkey = cv.take<uint64_t>(O);
    w.tsrc = cv.take<int>(O);
    w.tgr = cv.take<int>(O);
    w.tpl = cv.take<int>(O);
    w.tp1 = cv.take<float>(O);
    w.tp2 = cv.take<float>(O);
    return cv.size();
}

extern "C" size_t laue_simulate_workspace_size(const laue_geometry *geom, int32_t n_planes,
                                               int32_t n_grains, int64_t n_true_max,
                                               int64_t n_obs_max) {
    if (!geom || validate_geometry(geom) != LAUE_OK || n_grains < 0 || n_planes < 0) return 0;
    Carver cv(nullptr);
    SimWs w;
    return carve_sim(cv, w, geom, n_grains, n_true_max, n_obs_max, n_planes);
}

extern "C" int laue_simulate(const laue_geometry *geom, const laue_planes *planes,
                             const laue_grains *truth, double sigma_mm, double distance,
                             double outlier_frac, uint64_t seed, int64_t n_true_max,
                             float *p1, float *p2, int32_t *grain, int32_t *plane,
                             int64_t *block_off, int64_t *n_out, void *ws, size_t ws_bytes,
                             void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_geometry(geom)) || (rc = validate_planes(planes)) ||
        (rc = validate_grains(truth)))
        return rc;
    LAUE_REQUIRE(n_out && block_off, LAUE_EINVAL, "n_out or block_off is NULL");
    LAUE_REQUIRE(std::isfinite(sigma_mm) && sigma_mm >= 0 && std::isfinite(distance) && distance > 0,
                 LAUE_EINVAL, "sigma must be >= 0 and distance > 0");
    LAUE_REQUIRE(std::isfinite(outlier_frac) && outlier_frac >= 0 && outlier_frac <= 100,
                 LAUE_EINVAL, "bad outlier fraction");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t cap = *n_out;
    Carver cv(ws);
    SimWs w;
    size_t need = carve_sim(cv, w, geom, truth->n, n_true_max, cap, planes->n);
    if ((rc = check_ws(ws, ws_bytes, need))) return rc;
    std::vector<int64_t> sb;
    int64_t S = 0;
    if ((rc = enumerate_count(geom, planes, truth, 1, w.e, sb, &S, s))) return rc;
    if (S > n_true_max) {
        *n_out = -S;
        set_error("n_true_max " + std::to_string(n_true_max) + " < visible spots " + std::to_string(S));
        return LAUE_ECAPACITY;
    }
    const int nb = geom->n_rot * geom->n_det;
    const uint32_t k0 = static_cast<uint32_t>(seed & 0xffffffffu), k1 = static_cast<uint32_t>(seed >> 32);
    std::vector<int> nt(nb, 0), no(nb, 0);
    if (S > 0) {
        if ((rc = launch_enumerate_ids(geom, planes, w.e, truth->n, 1, S, w.plane, w.grain, w.block, s))) return rc;
        k_sim_noise<<<static_cast<unsigned>((S + 255) / 256), 256, 0, s>>>(
            *geom, planes->w, truth->q, truth->x, w.plane, w.grain, w.block, S, sigma_mm / distance,
            k0, k1, w.np1, w.np2, w.keep, w.key);
        LAUE_CHECK_HIP(hipGetLastError());
        k_sim_count<<<nb, 256, 0, s>>>(w.e.blk, w.keep, w.n_true);
        LAUE_CHECK_HIP(hipGetLastError());
        LAUE_CHECK_HIP(hipMemcpyAsync(nt.data(), w.n_true, nb * sizeof(int), hipMemcpyDeviceToHost, s));
        LAUE_CHECK_HIP(hipStreamSynchronize(s));
    }
    std::vector<int64_t> ob(nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
        no[b] = static_cast<int>(std::floor(outlier_frac * nt[b] + 0.5));
        ob[b + 1] = ob[b] + nt[b] + no[b];
    }
    const int64_t total = ob[nb];
    *n_out = total;
    std::memcpy(block_off, ob.data(), (nb + 1) * sizeof(int64_t));
    if (total > cap) {
        set_error("observed-spot capacity " + std::to_string(cap) + " < required " + std::to_string(total));
        return LAUE_ECAPACITY;
    }
    if (total == 0) return LAUE_OK;
    LAUE_REQUIRE(p1 && p2 && grain && plane, LAUE_EINVAL, "output arrays are NULL");
    LAUE_CHECK_HIP(hipMemcpyAsync(w.n_out, no.data(), nb * sizeof(int), hipMemcpyHostToDevice, s));
    LAUE_CHECK_HIP(hipMemcpyAsync(w.oblk, ob.data(), (nb + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    k_sim_emit<<<nb, 256, 0, s>>>(*geom, w.e.blk, w.keep, w.np1, w.np2, w.key, w.plane, w.grain,
                                   w.oblk, w.n_out, k0, k1, w.tkey, w.tsrc, w.tp1, w.tp2, w.tgr,
                                   w.tpl, p1, p2, grain, plane);
    LAUE_CHECK_HIP(hipGetLastError());
    LAUE_CHECK_HIP(hipStreamSynchronize(s));
    return LAUE_OK;
}
