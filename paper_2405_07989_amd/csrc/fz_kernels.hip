// fz_kernels.hip -- HIP kernels of libfz for gfx950 (CDNA4, wave64).
//
//   fz_dp_kernel        count table S[k][v] (completions of a prefix)
//   fz_restab_kernel    first element of the last-pair progression per
//                       residue class of the remainder modulo g[d-1]
//   fz_slices_kernel    rank-balanced slice bounds (Sec. 4 bounds, cut by rank)
//   fz_enum_kernel      the walker: bounded lexicographic enumeration with a
//                       count / length-histogram / predicate / store consumer
//   fz_finalize_kernel  sums, the slice self-check, histogram reduction
//   fz_unrank_kernel    element of a given rank (the fz_unrank entry point)
//
// Layout and notation are described in fz_internal.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fz_internal.h"

namespace {

__device__ __forceinline__ uint64_t sat_add(uint64_t x, uint64_t y)
{
    uint64_t s = x + y;
    return s < x ? ~0ull : s;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t x, const FzFastDiv &f)
{
    uint32_t t = __umulhi(f.m, x);
    return (t + ((x - t) >> f.s1)) >> f.s2;
}

// A lane's 64-bit value read by the whole wave (a wave-uniform result).
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane)
{
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t uni(uint32_t x)
{
    return __builtin_amdgcn_readfirstlane(x);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, uint32_t lane)
{
#pragma unroll
    for (int o = 1; o < FZK_WAVE; o <<= 1) {
        uint32_t t = __shfl_up(v, o, FZK_WAVE);
        if (lane >= (uint32_t)o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v, uint32_t lane)
{
#pragma unroll
    for (int o = 1; o < FZK_WAVE; o <<= 1) {
        uint64_t t = __shfl_up(v, o, FZK_WAVE);
        if (lane >= (uint32_t)o) v += t;
    }
    return v;
}

// Sum of a per-lane 64-bit value over the wave, returned to every lane as a
// wave-uniform value.
__device__ __forceinline__ uint64_t wave_sum64(uint64_t v)
{
#pragma unroll
    for (int o = FZK_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, FZK_WAVE);
    return readlane64(v, 0);
}

// S[d-1][v] = [g[d-1] divides v]; rows 0..d-2 are stored.
__device__ __forceinline__ uint64_t table_below(const FzPlan &P, const uint64_t *S, uint32_t k,
                                                uint32_t v)
{
    if (k + 1 == P.d - 1) return (v - fdiv(v, P.div_B) * P.B) == 0 ? 1ull : 0ull;
    return S[(uint64_t)(k + 1) * P.stride + v];
}

// Largest t in [0, v / gk] with Srow[v] - Srow[v - t gk] <= r: the number of
// completions with a_k < t is Srow[v] - Srow[v - t gk] (a telescoping sum of
// the next row), so t is the value of a_k at rank r.  r is reduced in place.
__device__ __forceinline__ uint32_t unrank_level(const uint64_t *Srow, uint32_t v, uint32_t gk,
                                                 uint64_t &r)
{
    const uint64_t sv = Srow[v];
    uint32_t lo = 0, hi = v / gk;
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo + 1) / 2;
        if (sv - Srow[v - mid * gk] <= r) lo = mid;
        else hi = mid - 1;
    }
    r -= sv - Srow[v - lo * gk];
    return lo;
}

} // namespace

// ---------------------------------------------------------------------------
// Count and work tables.  S[k][v] = #{(a_k..a_{d-1}) >= 0 : sum_{j>=k} a_j g_j
// = v} satisfies S[k][v] = S[k+1][v] + S[k][v - g_k]: along each chain
// v = c, c + g_k, c + 2 g_k, ... row k is the running sum of row k+1.  The
// work table C models what a wave pays: C[M][v] is the work of one row with
// remainder v (row_work), and C[k][v] = C[k+1][v] + C[k][v - g_k] sums it
// over the subtrees, so slices can be cut to equal work.
// One workgroup builds all rows; a row is g_k independent chains, each cut
// into row blocks (partial sums, a carry scan, then the final pass).
// Saturating adds: S[0][n] = 2^64-1 flags overflow.
// ---------------------------------------------------------------------------
// Work of the first t lanes (x = 0..t-1) of a row with remainder v: the row
// itself, its 64-lane chunks and its elements.  t = floor(v / G2) + 1 is the
// whole row.  Non-decreasing in t.
__device__ __forceinline__ uint64_t row_work(const FzPlan &P, const uint64_t *SM, uint32_t v,
                                             uint32_t t)
{
    if (t == 0) return 0;
    const uint64_t el = SM[v] - (t * (uint64_t)P.G2 <= v ? SM[v - t * P.G2] : 0);
    const uint64_t chunks = (t + FZK_WAVE - 1) / FZK_WAVE;
    uint64_t w = P.w_row + chunks * P.w_chunk;
    const uint64_t we = el * P.w_el;
    return (P.w_el && we / P.w_el != el) ? ~0ull : sat_add(w, we);
}

template <class Below>
__device__ void chain_scan(const FzPlan &P, uint64_t *row, uint32_t gk, Below below,
                           uint64_t *part)
{
    const uint32_t T = blockDim.x, tid = threadIdx.x;
    const uint32_t rows = P.n / gk + 1;
    const uint32_t cols = gk < P.stride ? gk : P.stride;
    const uint32_t nb = cols >= T ? 1 : T / cols;
    const uint32_t rpb = (rows + nb - 1) / nb;
    const uint32_t units = cols * nb;
    if (nb > 1) {
        for (uint32_t u = tid; u < units; u += T) {
            const uint32_t c = u % cols, b = u / cols;
            const uint32_t i1 = min(rows, (b + 1) * rpb);
            uint64_t s = 0;
            // independent loads first, then the dependent sum
            for (uint32_t i = b * rpb; i < i1; i += 8) {
                uint64_t x[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const uint64_t v = (uint64_t)(i + q) * gk + c;
                    x[q] = (i + q < i1 && v <= P.n) ? below((uint32_t)v) : 0;
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) s = sat_add(s, x[q]);
            }
            part[u] = s;
        }
        __syncthreads();
        for (uint32_t c = tid; c < cols; c += T) {
            uint64_t carry = 0;
            for (uint32_t b = 0; b < nb; ++b) {
                const uint64_t t = part[b * cols + c];
                part[b * cols + c] = carry;
                carry = sat_add(carry, t);
            }
        }
        __syncthreads();
    }
    for (uint32_t u = tid; u < units; u += T) {
        const uint32_t c = u % cols, b = u / cols;
        const uint32_t i1 = min(rows, (b + 1) * rpb);
        uint64_t run = nb > 1 ? part[u] : 0;
        for (uint32_t i = b * rpb; i < i1; i += 8) {
            uint64_t x[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint64_t v = (uint64_t)(i + q) * gk + c;
                x[q] = (i + q < i1 && v <= P.n) ? below((uint32_t)v) : 0;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint64_t v = (uint64_t)(i + q) * gk + c;
                run = sat_add(run, x[q]);
                if (i + q < i1 && v <= P.n) row[v] = run;
            }
        }
    }
    __syncthreads();
}

__global__ void __launch_bounds__(1024) fz_dp_kernel(FzPlan P, FzBufs Bf)
{
    __shared__ uint64_t part[1024];
    uint64_t *S = Bf.S;
    for (int k = (int)P.d - 2; k >= 0; --k) {
        uint64_t *row = S + (uint64_t)k * P.stride;
        const uint64_t *nxt = S + (uint64_t)(k + 1) * P.stride;
        if (k + 1 == (int)P.d - 1)
            chain_scan(P, row, P.g[k],
                       [&](uint32_t v) { return (v - fdiv(v, P.div_B) * P.B) == 0 ? 1ull : 0ull; },
                       part);
        else
            chain_scan(P, row, P.g[k], [&](uint32_t v) { return nxt[v]; }, part);
    }
    const int M = (int)P.d - 3;
    uint64_t *CM = Bf.C + (uint64_t)M * P.stride;
    const uint64_t *SM = S + (uint64_t)M * P.stride;
    for (uint32_t v = threadIdx.x; v <= P.n; v += blockDim.x)
        CM[v] = row_work(P, SM, v, fdiv(v, P.div_G2) + 1);
    __syncthreads();
    for (int k = M - 1; k >= 0; --k) {
        uint64_t *row = Bf.C + (uint64_t)k * P.stride;
        const uint64_t *nxt = Bf.C + (uint64_t)(k + 1) * P.stride;
        chain_scan(P, row, P.g[k], [&](uint32_t v) { return nxt[v]; }, part);
    }
}

// ---------------------------------------------------------------------------
// Residue table for the last pair (A, B) = (g[d-2], g[d-1]).  For a remainder
// rem = q B + rho the valid a[d-2] are t = t0 + j ord (j >= 0) with
// A t0 == rho (mod B), 0 <= t0 < ord; then a[d-1] = q - E - j delta with
// E = (A t0 - rho) / B.  Classes with gcd(A,B) not dividing rho have no
// element: E = FZK_NONE_E makes a[d-1] negative.  The table is doubled so
// that a lane can index it with rho' = rho + B in [0, 2B) and quotient
// q' = q - 1 without a borrow: entry rho' >= B holds E(rho' - B) - 1.
// ---------------------------------------------------------------------------
__global__ void fz_restab_kernel(FzPlan P, FzBufs Bf)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * P.B) return;
    const uint32_t rho = i < P.B ? i : i - P.B;
    int2 e;
    if (rho % P.D != 0) {
        e.x = 0;
        e.y = FZK_NONE_E;
    } else {
        const uint64_t t0 = ((uint64_t)(rho / P.D) * P.inv) % P.ord;
        const uint64_t num = (uint64_t)P.A * t0 - rho;
        e.x = (int)t0;
        e.y = (int)(num / P.B);
        if (i >= P.B) e.y -= 1;
    }
    Bf.restab[i] = e;
}

// ---------------------------------------------------------------------------
// Slice bounds, cut by work.  Lane prefixes a[0..M] in lex order carry the
// work of the wave that walks them (row_work).  Boundary j (0 <= j < W) is
// the prefix at work rank floor(j Wtot / W): found level by level in the work
// table for the row prefix a[0..M-1], then inside the row on the row_work of
// its first t lanes.  Wtot covers the prefixes up to the one that holds
// element rank N' - 1, N' = min(|Z|, max_tuples).  Slice j walks prefixes
// [bound j, bound j+1); base[j] is the element rank of its first element.
// Boundary W is open (sentinel).  Thread 0 also resets the control block.
// ---------------------------------------------------------------------------
__global__ void fz_slices_kernel(FzPlan P, FzBufs Bf)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t W = P.n_slices;
    const uint32_t np = P.d - 2;
    const uint32_t M = P.d - 3;
    const uint64_t N = Bf.S[P.n];
    const bool ovf = (N == ~0ull) || (Bf.C[P.n] == ~0ull);
    if (j == 0) {
        FzCtl *c = Bf.ctl;
        c->cursor = 0;
        c->found = 0;
        c->status = ovf ? FZS_OVERFLOW : 0u;
        c->total = N;
        c->count = 0;
        c->rows = 0;
        c->prefixes = 0;
        c->written = 0;
    }
    if (j > W) return;
    const uint64_t Np = ovf ? 0 : (N < P.max_tuples ? N : P.max_tuples);
    uint32_t *out = Bf.bounds + (uint64_t)j * np;
    if (j == W || Np == 0) {
        Bf.base[j] = Np;
        out[0] = FZK_SENTINEL;
        return;
    }
    const uint64_t *SM = Bf.S + (uint64_t)M * P.stride;
    uint64_t Wtot;
    if (Np == N) {
        Wtot = Bf.C[P.n];
    } else {
        // work of the rows before the one that holds element rank Np-1, plus
        // that row up to and including the lane holding it
        uint64_t r = Np - 1, acc = 0;
        uint32_t v = P.n;
        for (uint32_t k = 0; k < M; ++k) {
            const uint64_t *Ck = Bf.C + (uint64_t)k * P.stride;
            const uint32_t t = unrank_level(Bf.S + (uint64_t)k * P.stride, v, P.g[k], r);
            acc += Ck[v] - Ck[v - t * P.g[k]];
            v -= t * P.g[k];
        }
        const uint32_t x = unrank_level(SM, v, P.G2, r);
        Wtot = acc + row_work(P, SM, v, x + 1);
    }
    uint64_t rc = (Wtot / W) * j + ((Wtot % W) * j) / W;
    uint64_t base = 0;
    uint32_t v = P.n;
    for (uint32_t k = 0; k < M; ++k) {
        const uint64_t *Sk = Bf.S + (uint64_t)k * P.stride;
        const uint32_t t = unrank_level(Bf.C + (uint64_t)k * P.stride, v, P.g[k], rc);
        base += Sk[v] - Sk[v - t * P.g[k]];
        out[k] = t;
        v -= t * P.g[k];
    }
    // inside the row: largest t in [0, v / G2] whose first t lanes fit in rc
    uint32_t lo = 0, hi = v / P.G2;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo + 1) / 2;
        if (row_work(P, SM, v, mid) <= rc) lo = mid;
        else hi = mid - 1;
    }
    out[M] = lo;
    base += SM[v] - SM[v - lo * P.G2];
    Bf.base[j] = base;
}

// ---------------------------------------------------------------------------
// The walker.  Persistent workgroups of four waves; each wave takes slices
// from an atomic cursor.  Within a slice the row prefix a[0..M-1] is a
// wave-uniform odometer in ascending lex order (scalar registers); a row is
// cut into chunks of 64 consecutive values of the lane coordinate x = a[M];
// each lane solves its last pair from the residue table and then steps its
// progression of elements one candidate at a time (the modulo skip of
// Sec. 3.2.4: a[d-2] += ord, a[d-1] -= delta), the step ending at the first
// candidate with a[d-1] < 0.  The consumer sees every element.
//
// LDS: [residue table, 2B int2, when it fits][per-wave consumer scratch].
// ---------------------------------------------------------------------------
template <int M, int MODE, bool TLDS>
__global__ void __launch_bounds__(FZK_WG) fz_enum_kernel(FzPlan P, FzBufs Bf)
{
    extern __shared__ __align__(16) uint32_t lds[];
    constexpr uint32_t NP = M + 1;
    const uint32_t lane = __lane_id();
    const uint32_t wave = threadIdx.x / FZK_WAVE;
    const uint32_t W = P.n_slices;

    // TLDS: the residue table is staged in LDS (read with ds_read); else it
    // is read from global memory.  Two instantiations keep each pointer's
    // address space known to the compiler.
    int2 *ltab = (int2 *)lds;
    uint32_t *scratch = lds;
    if constexpr (TLDS) {
        for (uint32_t i = threadIdx.x; i < 2 * P.B; i += blockDim.x) ltab[i] = Bf.restab[i];
        scratch = lds + 2 * (((2 * P.B) + 1) & ~1u); // keep 16-byte alignment
    }
    uint32_t *wbins = nullptr;
    uint64_t *grow = nullptr;
    if constexpr (MODE == FZM_HIST) {
        if (P.hist_in_lds) {
            wbins = scratch + wave * (P.nbins + FZK_WAVE);
            for (uint32_t i = lane; i < P.nbins + FZK_WAVE; i += FZK_WAVE) wbins[i] = 0;
            grow = Bf.hist_rows + (uint64_t)blockIdx.x * P.nbins;
            for (uint32_t i = threadIdx.x; i < P.nbins; i += blockDim.x) grow[i] = 0;
        }
    }
    // store scratch per wave: scan (64 x u64), t0 and ad0 (64 x u32 each),
    // then the staging block of 64 rows x d_user words
    const uint32_t store_words = 4 * FZK_WAVE + FZK_WAVE * P.d_user;
    uint64_t *s_incl = (uint64_t *)(scratch + wave * store_words);
    uint32_t *s_t0 = (uint32_t *)(s_incl + FZK_WAVE);
    uint32_t *s_ad0 = s_t0 + FZK_WAVE;
    uint32_t *s_stage = s_ad0 + FZK_WAVE;
    __syncthreads();

    // lane * G2 = lq * B + lr (exact whenever the lane is active).  A lane
    // reads the doubled residue table at rho' = Pc + (B - lr) with quotient
    // q' = Qc - (lq + 1): no borrow to propagate.
    const uint64_t lg = (uint64_t)lane * P.G2;
    const uint32_t lq1 = (uint32_t)(lg / P.B) + 1;
    const uint32_t lr2 = P.B - (uint32_t)(lg % P.B);
    const uint32_t len_step = P.ord - P.delta;
    const int32_t delta = (int32_t)P.delta;
    uint64_t hist_since_flush = 0;

    // The spine of this loop must stay free of lane-dependent branches: every
    // lane takes part in the cursor atomic (only lane 0 adds 1) and every lane
    // stores the same slice record, so the wave walks each slice as a whole.
    for (;;) {
        const uint32_t old = atomicAdd(&Bf.ctl->cursor, lane == 0 ? 1u : 0u);
        const uint32_t s = __builtin_amdgcn_readlane(old, 0);
        if (s >= W) break;
        if constexpr (MODE == FZM_EXISTS) {
            const uint32_t f =
                __hip_atomic_load(&Bf.ctl->found, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (uni(f)) break;
        }
        const uint64_t t_begin = wall_clock64();
        const uint32_t *b0 = Bf.bounds + (uint64_t)s * NP;
        const uint32_t *b1 = b0 + NP;
        // per-lane element counters: a chunk adds at most n + 1 per lane to
        // the 32-bit counter, which is folded into the 64-bit one per chunk
        uint64_t lane_el = 0;
        uint32_t lane_pref = 0;
        uint64_t n_el = 0, n_rows = 0;
        if (uni(b0[0]) != FZK_SENTINEL) {
            uint32_t a[M > 0 ? M : 1];
            uint32_t e[M > 0 ? M : 1];
            uint32_t rr[M + 1]; // rr[k]: remainder after a[0..k-1]
            rr[0] = P.n;
#pragma unroll
            for (int k = 0; k < M; ++k) {
                a[k] = uni(b0[k]);
                rr[k + 1] = rr[k] - a[k] * P.g[k];
            }
            int32_t xs = (int32_t)uni(b0[M]);
            const bool end_open = uni(b1[0]) == FZK_SENTINEL;
            int32_t xe = 0;
#pragma unroll
            for (int k = 0; k < M; ++k) e[k] = 0;
            if (!end_open) {
#pragma unroll
                for (int k = 0; k < M; ++k) e[k] = uni(b1[k]);
                xe = (int32_t)uni(b1[M]);
            }
            uint32_t plen = 0;
#pragma unroll
            for (int k = 0; k < M; ++k) plen += a[k];
            uint64_t rank = Bf.base[s];
            bool done = false;
            while (!done) {
                const uint32_t Rp = rr[M];
                const int32_t xhi = (int32_t)fdiv(Rp, P.div_G2);
                bool last = !end_open;
#pragma unroll
                for (int k = 0; k < M; ++k) last = last && (a[k] == e[k]);
                const int32_t xlast = last ? xe - 1 : xhi;
                ++n_rows;
                if constexpr (MODE == FZM_EXISTS) {
                    const uint32_t f = __hip_atomic_load(&Bf.ctl->found, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                    if (uni(f)) break;
                }
                for (int32_t c = xs; c <= xlast; c += FZK_WAVE) {
                    const uint32_t Rc = Rp - (uint32_t)c * P.G2;
                    const uint32_t Qc = fdiv(Rc, P.div_B);
                    const uint32_t Pc = Rc - Qc * P.B;
                    const bool active = (int32_t)lane <= xlast - c;
                    const uint32_t rho2 = Pc + lr2;
                    const int32_t q2 = (int32_t)(Qc - lq1);
                    const uint32_t ti = active ? rho2 : 0u;
                    const int2 ent = TLDS ? ltab[ti] : Bf.restab[ti];
                    // a lane with no element starts at -1, so that the common
                    // decrement stays above -(n + 2 A) > -2^31 for every lane
                    int32_t ad0 = q2 - ent.y;
                    ad0 = (active && ad0 >= 0) ? ad0 : -1;
                    lane_pref += active ? 1u : 0u;
                    uint32_t cnt = 0;
                    if constexpr (MODE == FZM_COUNT) {
                        // two candidate steps per trip; the trip test is the
                        // first step's own validity test
                        int32_t ad = ad0;
                        for (;;) {
                            const bool c0 = ad >= 0;
                            if (!__ballot(c0)) break;
                            const bool c1 = ad >= delta;
                            cnt += c0 ? 1u : 0u;
                            cnt += c1 ? 1u : 0u;
                            ad -= 2 * delta;
                        }
                        lane_el += cnt;
                    } else if constexpr (MODE == FZM_HIST) {
                        int32_t ad = ad0;
                        uint32_t len = plen + (uint32_t)c + lane + (uint32_t)ent.x + (uint32_t)ad0;
                        uint64_t *gh = Bf.hist;
                        // lanes without an element add into a private spare bin
                        const uint32_t spare = P.nbins + lane;
                        for (;;) {
                            const bool c0 = ad >= 0;
                            if (!__ballot(c0)) break;
                            cnt += c0 ? 1u : 0u;
                            if (P.hist_in_lds) {
                                atomicAdd(&wbins[c0 ? len : spare], 1u);
                            } else if (c0) {
                                atomicAdd((unsigned long long *)&gh[len], 1ull);
                            }
                            ad -= delta;
                            len += len_step;
                        }
                        lane_el += cnt;
                    } else if constexpr (MODE == FZM_EXISTS) {
                        int32_t ad = ad0;
                        uint32_t len = plen + (uint32_t)c + lane + (uint32_t)ent.x + (uint32_t)ad0;
                        bool hit = false;
                        for (;;) {
                            const bool c0 = ad >= 0;
                            if (!__ballot(c0)) break;
                            cnt += c0 ? 1u : 0u;
                            if (__ballot(c0 && (uint64_t)len == P.target_len)) {
                                hit = true;
                                break;
                            }
                            ad -= delta;
                            len += len_step;
                        }
                        lane_el += cnt;
                        if (hit) {
                            __hip_atomic_store(&Bf.ctl->found, 1u, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                            done = true;
                            break;
                        }
                    } else { // FZM_STORE
                        uint64_t L = 0;
                        if (ad0 >= 0) L = fdiv((uint32_t)ad0, P.div_delta) + 1;
                        const uint64_t incl = wave_incl_scan64(L, lane);
                        const uint64_t T = readlane64(incl, FZK_WAVE - 1);
                        s_incl[lane] = incl;
                        s_t0[lane] = (uint32_t)ent.x;
                        s_ad0[lane] = (uint32_t)ad0;
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                        // Rows are produced 64 at a time (lane = position in
                        // the chunk's output), staged in LDS as one
                        // contiguous block and written out as consecutive
                        // dwords: every store instruction covers 256 bytes.
                        const uint64_t lim = P.max_tuples;
                        const uint32_t du = P.d_user;
                        for (uint64_t p0 = 0; p0 < T && rank + p0 < lim; p0 += FZK_WAVE) {
                            const uint64_t left = T - p0 < lim - rank - p0 ? T - p0 : lim - rank - p0;
                            const uint32_t nb = left < FZK_WAVE ? (uint32_t)left : FZK_WAVE;
                            const uint64_t p = p0 + lane;
                            if (lane < nb) {
                                uint32_t j = 0;
#pragma unroll
                                for (uint32_t st = FZK_WAVE / 2; st >= 1; st >>= 1)
                                    if (s_incl[j + st - 1] <= p) j += st;
                                const uint32_t k = (uint32_t)(p - (j ? s_incl[j - 1] : 0ull));
                                uint32_t v[M + 3];
#pragma unroll
                                for (int q = 0; q < M; ++q) v[q] = a[q];
                                v[M] = (uint32_t)c + j;
                                v[M + 1] = s_t0[j] + k * P.ord;
                                v[M + 2] = s_ad0[j] - k * P.delta;
                                uint32_t *st_row = s_stage + lane * du - P.pad;
#pragma unroll
                                for (int q = 0; q < M + 3; ++q)
                                    if ((uint32_t)q >= P.pad) st_row[q] = v[q];
                            }
                            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                            __builtin_amdgcn_wave_barrier();
                            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                            uint32_t *dst = Bf.out + (rank + p0) * du;
                            const uint32_t words = nb * du;
                            for (uint32_t i = lane; i < words; i += FZK_WAVE) dst[i] = s_stage[i];
                            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                            __builtin_amdgcn_wave_barrier();
                            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                        }
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                        if (rank < lim) n_el += (T < lim - rank) ? T : (lim - rank);
                        rank += T;
                        if (rank >= lim) {
                            done = true;
                            break;
                        }
                    }
                }
                if (done || last) break;
                // next row: rightmost k whose a[k] can grow, deeper coordinates reset
                int kk = -1;
#pragma unroll
                for (int k = 0; k < M; ++k)
                    if (rr[k + 1] >= P.g[k]) kk = k;
                if (kk < 0) break;
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    if (k == kk) {
                        a[k] += 1;
                        rr[k + 1] -= P.g[k];
                    } else if (k > kk) {
                        a[k] = 0;
                        rr[k + 1] = rr[k];
                    }
                }
                plen = 0;
#pragma unroll
                for (int k = 0; k < M; ++k) plen += a[k];
                xs = 0;
            }
        }
        if constexpr (MODE != FZM_STORE) n_el = wave_sum64(lane_el);
        {
            FzSliceRec rec;
            rec.elements = n_el;
            rec.rows = n_rows;
            rec.prefixes = wave_sum64(lane_pref);
            rec.t_begin = t_begin;
            rec.t_end = wall_clock64();
            Bf.recs[s] = rec; // the same value from every lane
        }
        if constexpr (MODE == FZM_HIST) {
            hist_since_flush += n_el;
            if (P.hist_in_lds && hist_since_flush > (1ull << 31)) {
                for (uint32_t i = lane; i < P.nbins; i += FZK_WAVE) {
                    const uint32_t h = wbins[i];
                    if (h) {
                        atomicAdd((unsigned long long *)&grow[i], (unsigned long long)h);
                        wbins[i] = 0;
                    }
                }
                hist_since_flush = 0;
            }
        }
    }
    if constexpr (MODE == FZM_HIST) {
        if (P.hist_in_lds) {
            for (uint32_t i = lane; i < P.nbins; i += FZK_WAVE) {
                const uint32_t h = wbins[i];
                if (h) atomicAdd((unsigned long long *)&grow[i], (unsigned long long)h);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Finalize: element / row / prefix totals, the slice self-check (each slice
// must have produced exactly the ranks between its bound and the next), the
// reduction of the per-workgroup histograms, and min / max length.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) fz_finalize_kernel(FzPlan P, FzBufs Bf, uint32_t nwg)
{
    __shared__ uint64_t red[4][1024 / FZK_WAVE];
    const uint32_t tid = threadIdx.x, lane = tid % FZK_WAVE, w = tid / FZK_WAVE;
    const uint32_t nw = blockDim.x / FZK_WAVE;
    uint64_t el = 0, rows = 0, pref = 0, bad = 0;
    for (uint32_t s = tid; s < P.n_slices; s += blockDim.x) {
        const FzSliceRec r = Bf.recs[s];
        el += r.elements;
        rows += r.rows;
        pref += r.prefixes;
        if (P.mode != FZM_EXISTS && r.elements != Bf.base[s + 1] - Bf.base[s]) bad = 1;
    }
    uint64_t lo = ~0ull, hi = 0;
    if (P.mode == FZM_HIST) {
        for (uint32_t l = tid; l < P.nbins; l += blockDim.x) {
            uint64_t h;
            if (P.hist_in_lds) {
                h = 0;
                for (uint32_t b = 0; b < nwg; ++b) h += Bf.hist_rows[(uint64_t)b * P.nbins + l];
                Bf.hist[l] = h;
            } else {
                h = Bf.hist[l];
            }
            if (h) {
                lo = l < lo ? l : lo;
                hi = l > hi ? l : hi;
            }
        }
    }
    for (int o = FZK_WAVE / 2; o > 0; o >>= 1) {
        el += __shfl_xor(el, o);
        rows += __shfl_xor(rows, o);
        pref += __shfl_xor(pref, o);
        bad |= __shfl_xor(bad, o);
        const uint64_t lo2 = __shfl_xor(lo, o), hi2 = __shfl_xor(hi, o);
        lo = lo2 < lo ? lo2 : lo;
        hi = hi2 > hi ? hi2 : hi;
    }
    __shared__ uint64_t mm[2][1024 / FZK_WAVE];
    if (lane == 0) {
        red[0][w] = el;
        red[1][w] = rows;
        red[2][w] = pref;
        red[3][w] = bad;
        mm[0][w] = lo;
        mm[1][w] = hi;
    }
    __syncthreads();
    if (tid == 0) {
        uint64_t t[4] = {0, 0, 0, 0};
        uint64_t L = ~0ull, H = 0;
        for (uint32_t i = 0; i < nw; ++i) {
            for (int q = 0; q < 4; ++q) t[q] = (q == 3) ? (t[q] | red[q][i]) : t[q] + red[q][i];
            L = mm[0][i] < L ? mm[0][i] : L;
            H = mm[1][i] > H ? mm[1][i] : H;
        }
        FzCtl *c = Bf.ctl;
        c->count = t[0];
        c->rows = t[1];
        c->prefixes = t[2];
        if (t[3]) c->status |= FZS_MISMATCH;
        c->min_len = L;
        c->max_len = H;
        const uint64_t N = c->total;
        c->written = (c->status & FZS_OVERFLOW) ? 0 : (N < P.max_tuples ? N : P.max_tuples);
    }
}

// ---------------------------------------------------------------------------
// Element of each requested rank (fz_unrank): the slice-bound search carried
// through all d coordinates.  A rank >= |Z| sets FZS_MISMATCH and leaves its
// row untouched.
// ---------------------------------------------------------------------------
__global__ void fz_unrank_kernel(FzPlan P, FzBufs Bf, const uint64_t *ranks, uint64_t nr,
                                 uint32_t *out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    const uint64_t N = Bf.S[P.n];
    uint64_t r = ranks[i];
    if (N == ~0ull || r >= N) {
        atomicOr(&Bf.ctl->status, FZS_MISMATCH);
        return;
    }
    uint32_t v = P.n;
    uint32_t *dst = out + i * P.d_user - P.pad;
    for (uint32_t k = 0; k + 1 < P.d; ++k) {
        const uint32_t t = unrank_level(Bf.S + (uint64_t)k * P.stride, v, P.g[k], r);
        if (k >= P.pad) dst[k] = t;
        v -= t * P.g[k];
    }
    dst[P.d - 1] = v / P.B;
}

__global__ void fz_zero_kernel(uint64_t *p, uint64_t count)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
hipError_t fzk_launch_dp(const FzPlan &p, const FzBufs &b, hipStream_t s)
{
    hipLaunchKernelGGL(fz_dp_kernel, dim3(1), dim3(1024), 0, s, p, b);
    return hipGetLastError();
}

hipError_t fzk_launch_restab(const FzPlan &p, const FzBufs &b, hipStream_t s)
{
    const uint32_t blocks = (2 * p.B + 255) / 256;
    hipLaunchKernelGGL(fz_restab_kernel, dim3(blocks), dim3(256), 0, s, p, b);
    return hipGetLastError();
}

hipError_t fzk_launch_slices(const FzPlan &p, const FzBufs &b, hipStream_t s)
{
    const uint32_t blocks = (p.n_slices + 1 + 255) / 256;
    hipLaunchKernelGGL(fz_slices_kernel, dim3(blocks), dim3(256), 0, s, p, b);
    if (p.mode == FZM_HIST && !p.hist_in_lds)
        hipLaunchKernelGGL(fz_zero_kernel, dim3(256), dim3(256), 0, s, b.hist, (uint64_t)p.nbins);
    return hipGetLastError();
}

size_t fzk_enum_lds_bytes(const FzPlan &p)
{
    const uint32_t waves = FZK_WG / FZK_WAVE;
    size_t bytes = p.restab_in_lds ? (size_t)2 * ((2 * p.B + 1) & ~1u) * sizeof(uint32_t) : 0;
    if (p.mode == FZM_HIST && p.hist_in_lds)
        bytes += (size_t)waves * (p.nbins + FZK_WAVE) * sizeof(uint32_t);
    if (p.mode == FZM_STORE)
        bytes += (size_t)waves * (4 * FZK_WAVE + FZK_WAVE * p.d_user) * sizeof(uint32_t);
    return bytes;
}

template <int M, bool TLDS>
static void launch_enum_mt(const FzPlan &p, const FzBufs &b, uint32_t nwg, hipStream_t s)
{
    const size_t lds = fzk_enum_lds_bytes(p);
    switch (p.mode) {
    case FZM_COUNT:
        hipLaunchKernelGGL((fz_enum_kernel<M, FZM_COUNT, TLDS>), dim3(nwg), dim3(FZK_WG), lds, s,
                           p, b);
        break;
    case FZM_HIST:
        hipLaunchKernelGGL((fz_enum_kernel<M, FZM_HIST, TLDS>), dim3(nwg), dim3(FZK_WG), lds, s,
                           p, b);
        break;
    case FZM_EXISTS:
        hipLaunchKernelGGL((fz_enum_kernel<M, FZM_EXISTS, TLDS>), dim3(nwg), dim3(FZK_WG), lds, s,
                           p, b);
        break;
    default:
        hipLaunchKernelGGL((fz_enum_kernel<M, FZM_STORE, TLDS>), dim3(nwg), dim3(FZK_WG), lds, s,
                           p, b);
        break;
    }
}

template <int M>
static hipError_t launch_enum_m(const FzPlan &p, const FzBufs &b, uint32_t nwg, hipStream_t s)
{
    if (p.restab_in_lds) launch_enum_mt<M, true>(p, b, nwg, s);
    else launch_enum_mt<M, false>(p, b, nwg, s);
    return hipGetLastError();
}

hipError_t fzk_launch_enum(const FzPlan &p, const FzBufs &b, uint32_t nwg, hipStream_t s)
{
    switch (p.d - 3) {
    case 0: return launch_enum_m<0>(p, b, nwg, s);
    case 1: return launch_enum_m<1>(p, b, nwg, s);
    case 2: return launch_enum_m<2>(p, b, nwg, s);
    case 3: return launch_enum_m<3>(p, b, nwg, s);
    case 4: return launch_enum_m<4>(p, b, nwg, s);
    case 5: return launch_enum_m<5>(p, b, nwg, s);
    case 6: return launch_enum_m<6>(p, b, nwg, s);
    case 7: return launch_enum_m<7>(p, b, nwg, s);
    case 8: return launch_enum_m<8>(p, b, nwg, s);
    case 9: return launch_enum_m<9>(p, b, nwg, s);
    case 10: return launch_enum_m<10>(p, b, nwg, s);
    case 11: return launch_enum_m<11>(p, b, nwg, s);
    case 12: return launch_enum_m<12>(p, b, nwg, s);
    case 13: return launch_enum_m<13>(p, b, nwg, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t fzk_launch_finalize(const FzPlan &p, const FzBufs &b, uint32_t nwg, hipStream_t s)
{
    hipLaunchKernelGGL(fz_finalize_kernel, dim3(1), dim3(1024), 0, s, p, b, nwg);
    return hipGetLastError();
}

hipError_t fzk_launch_unrank(const FzPlan &p, const FzBufs &b, const uint64_t *ranks,
                             uint64_t nranks, uint32_t *out, hipStream_t s)
{
    if (nranks == 0) return hipSuccess;
    const uint64_t blocks = (nranks + 255) / 256;
    hipLaunchKernelGGL(fz_unrank_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, p, b, ranks,
                       nranks, out);
    return hipGetLastError();
}
