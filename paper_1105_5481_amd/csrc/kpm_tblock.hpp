// Temporal blocking of the recursion on 2D lattices with real hopping: two
// steps per pass over the vectors.
//
// One pass reads r_{n-1} and r_n and writes r_{n+1} and r_{n+2}, 4 vector
// transfers for 2 steps instead of 6.  A work item is an x-tile of T sites
// times a segment of rows (the march axis y).  Its block holds a window of
// W = TB_BLOCK / C sites (T = W - 2h owned plus h halo sites on each side;
// h = 2, or the depth D of the solve's deeper passes, k_step_tbd), one
// thread per 16-byte chunk, and marches along y with rows y-1, y, y+1 of r_n
// and rows y-2, y-1 of r_{n+1} in registers; in-row neighbours come through
// LDS.  Row y of r_{n+1} is computed on the window minus its outer sites (the
// owned sites plus one halo site each side, recomputed by both neighbouring
// tiles), row y-1 of r_{n+2} on the owned sites.  Segment ends are handled the
// same way along y (one extra row of r_{n+1} each side).  Every value is formed
// with the one-step kernel's expression, so the vectors are bitwise equal to
// the one-step recursion's.
//
// The halo recomputation means r_{n-1} and r_n are read by neighbouring tiles
// while the pass runs, so the outputs go to the two free buffers of four: the
// host passes the four buffers (prev, cur, out1, out2) of every launch.
// Phase 0 writes r_0 (and the partials of <r_0|r_0>) into `cur`; phase 1 is a
// pair of steps n, n+1; phase 2 a single step n (the last of an odd count, or
// when the caller advances one step).  The loads of row y+1 are issued one row
// ahead, so their latency overlaps the two barriers of the current row;
// r_{n-1} (read once) and the outputs (written once) use non-temporal
// accesses when the instance streams.
#pragma once

namespace kpm {

constexpr int TB_BLOCK = 512;
constexpr int MODE_TB = 3;   // plan mode of solves run by this kernel

template <typename S, bool WIDE, bool NT>
__global__ __launch_bounds__(TB_BLOCK) void k_step_tb(const Inst *__restrict__ tab, int32_t n, int32_t phase,
                                                      const void *prev, void *cur, void *out1, void *out2)
{
    typedef typename V16<S>::T T;
    typedef Mem<S, WIDE> G;
    __shared__ T rn_s[TB_BLOCK];
    __shared__ T r1_s[2][TB_BLOCK];
    const Inst I = tab[0];
    const uint32_t C = I.C, Lx = I.P, Ly = I.Lm;
    const uint32_t h = (uint32_t)I.tbh, Wn = TB_BLOCK / C, Tn = Wn - 2 * h;
    const uint32_t tid = threadIdx.x, s = tid / C, c = tid - s * C;
    const bool hd = I.has_diag;
    const S hop = G::lds(I.hop, 0);
    const bool first = (n == 0), two = (phase == 1);
    typedef typename V16<S>::T Tv;
    const Tv zero = (Tv)(S)0;
    double *part1 = I.partial + (size_t)((phase == 0 ? 0 : n + 1) % I.pslots) * I.tiles * 4;
    double *part2 = I.partial + (size_t)((n + 2) % I.pslots) * I.tiles * 4;
    const ItemRange ir = item_range(I, I.nct, I.nseg);
    for (uint32_t it = ir.first; it < ir.count; it += ir.stride) {
        const uint32_t sl = it / ir.nu;
        const uint32_t sg = ir.sb + sl;
        const uint32_t tx = ir.ub + (it - sl * ir.nu);
        const uint32_t x0 = tx * Tn;
        const uint32_t xend = min(x0 + Tn, Lx);
        const uint32_t x = (x0 + Lx - h + s) % Lx;
        const bool own_x = s >= h && s < Wn - h && x0 + s - h < xend;
        const bool ring1 = s >= 1 && s + 1 < Wn;
        const uint32_t y0 = sg * I.S, y1 = min(y0 + I.S, Ly), ns = y1 - y0;
        const uint32_t t = sg * I.nct + tx;
        Dots<S> a1, a2;
        if (phase == 0) {
            if (own_x)
                for (uint32_t y = y0; y < y1; ++y) {
                    const uint32_t i = x + Lx * y;
                    const T v = start_chunk<S>(I, i, c);
                    G::st(cur, i * C + c, v);
                    a1.norm_only(v);
                }
            block_reduce_store<Dots<S>::DD, TB_BLOCK>(a1.s0, a1.c0, a1.s1, a1.c1, part1 + (size_t)t * 4);
            continue;
        }
        auto row = [&](uint32_t y0m, int32_t off) { return (y0m + Ly + (uint32_t)off) % Ly; };   // y0m + off, periodic
        uint32_t ya = row(y0, -2), yb = row(y0, -1);
        T rnm = G::ld(cur, (x + Lx * ya) * C + c);
        T rn0 = G::ld(cur, (x + Lx * yb) * C + c);
        S dm = hd ? G::lds(I.diag, x + Lx * ya) : (S)0;
        S d0 = hd ? G::lds(I.diag, x + Lx * yb) : (S)0;
        T r1m2 = zero, r1m1 = zero;
        // row y0 of r_n (and its diagonal) and row y0-1 of r_{n-1}, one row ahead
        T rnp_n = G::ld(cur, (x + Lx * y0) * C + c);
        S dp_n = hd ? G::lds(I.diag, x + Lx * y0) : (S)0;
        T pv_n = (ring1 && !first) ? G::template ld_s<NT>(prev, (x + Lx * yb) * C + c) : zero;
        for (uint32_t j = 0; j <= ns + 1; ++j) {
            const uint32_t y = row(y0, (int32_t)j - 1);
            const T rnp = rnp_n;
            const S dp = dp_n;
            const T pv = pv_n;
            if (j <= ns) {   // rows needed by the next iteration
                const uint32_t yn = row(y0, (int32_t)j + 1);
                rnp_n = G::ld(cur, (x + Lx * yn) * C + c);
                dp_n = hd ? G::lds(I.diag, x + Lx * yn) : (S)0;
                if (ring1 && !first) pv_n = G::template ld_s<NT>(prev, (x + Lx * row(y0, (int32_t)j)) * C + c);
            }
            rn_s[tid] = rn0;
            __syncthreads();
            T r1 = zero;
            if (ring1) {
                const T nb[4] = {rn_s[tid - C], rn_s[tid + C], rnm, rnp};
                r1 = apply_real<S, 4>(hd, d0, hop, rn0, nb);
                if (!first) r1 = (S)2 * r1 - pv;
            }
            if (own_x && j >= 1 && j <= ns) {
                G::template st_s<NT>(out1, (x + Lx * y) * C + c, r1);
                a1.add(r1, rn0);
            }
            r1_s[j & 1][tid] = r1;
            __syncthreads();
            if (two && own_x && j >= 2) {
                const T nb[4] = {r1_s[(j - 1) & 1][tid - C], r1_s[(j - 1) & 1][tid + C], r1m2, r1};
                T r2 = apply_real<S, 4>(hd, dm, hop, r1m1, nb);
                r2 = (S)2 * r2 - rnm;
                const uint32_t ym = row(y0, (int32_t)j - 2);
                G::template st_s<NT>(out2, (x + Lx * ym) * C + c, r2);
                a2.add(r2, r1m1);
            }
            r1m2 = r1m1;
            r1m1 = r1;
            rnm = rn0;
            rn0 = rnp;
            dm = d0;
            d0 = dp;
        }
        block_reduce_store<Dots<S>::DD, TB_BLOCK>(a1.s0, a1.c0, a1.s1, a1.c1, part1 + (size_t)t * 4);
        if (two) block_reduce_store<Dots<S>::DD, TB_BLOCK>(a2.s0, a2.c0, a2.s1, a2.c1, part2 + (size_t)t * 4);
    }
}

// Depth-D passes (D = 3 .. 6; solves whose x-tiles carry a halo of h >= D
// sites): one launch advances D steps.  It reads r_{n-1} and r_n and writes
// only r_{n+D-1} and r_{n+D}, all the next pass needs; r_{n+1} .. r_{n+D-2}
// exist only on chip, where their dots are formed: 4 vector transfers for D
// steps.  Level k = 1..D computes r_{n+k}; at iteration j (row
// y = y0 - (D-1) + j) level k handles row y - (k-1) on the sites at least k
// from the window edge (level D: the owned sites), from level k-1 at rows
// y - k .. y - k + 2 (level 0 = r_n, rows y - 1 .. y + 1) and level k-2 at
// row y - (k-1) (r_{n-1} for level 1).  In-row neighbours come through LDS,
// every level's row double-buffered so that one block barrier per row
// suffices; rows in registers otherwise.  Every value is formed with the
// one-step kernel's expression, so the vectors are bitwise those of one-step
// passes.
template <typename S, bool WIDE, bool NT, int D>
__global__ __launch_bounds__(TB_BLOCK) void k_step_tbd(const Inst *__restrict__ tab, int32_t n, const void *prev,
                                                       const void *cur, void *outa, void *outb)
{
    typedef typename V16<S>::T T;
    typedef Mem<S, WIDE> G;
    __shared__ T lv_s[D][2][TB_BLOCK];   // level k's row of the iteration, double-buffered (k < D)
    const Inst I = tab[0];
    const uint32_t C = I.C, Lx = I.P, Ly = I.Lm;
    const uint32_t h = (uint32_t)I.tbh, Wn = TB_BLOCK / C, Tn = Wn - 2 * h;   // h >= D
    const uint32_t tid = threadIdx.x, s = tid / C, c = tid - s * C;
    const bool hd = I.has_diag;
    const S hop = G::lds(I.hop, 0);
    const bool first = (n == 0);
    const T zero = (T)(S)0;
    const ItemRange ir = item_range(I, I.nct, I.nseg);
    for (uint32_t it = ir.first; it < ir.count; it += ir.stride) {
        const uint32_t sl = it / ir.nu;
        const uint32_t sg = ir.sb + sl;
        const uint32_t tx = ir.ub + (it - sl * ir.nu);
        const uint32_t x0 = tx * Tn;
        const uint32_t xend = min(x0 + Tn, Lx);
        const uint32_t x = (x0 + Lx - h + s) % Lx;
        const bool own = s >= h && s < Wn - h && x0 + s - h < xend;
        const uint32_t y0 = sg * I.S, y1 = min(y0 + I.S, Ly), ns = y1 - y0;
        const uint32_t t = sg * I.nct + tx;
        Dots<S> acc[D];
        auto row = [&](int32_t off) { return (y0 + Ly + (uint32_t)off) % Ly; };   // y0 + off, periodic
        // level 0 (r_n): rows y-1, y, y+1 of the current iteration; diagonal d[q] of row y + 1 - q
        T rnm = G::ld(cur, (x + Lx * row(-D)) * C + c);
        T rn0 = G::ld(cur, (x + Lx * row(1 - D)) * C + c);
        S d[D + 2];
#pragma unroll
        for (int q = 0; q < D + 2; ++q) d[q] = (S)0;
        if (hd) {
            d[2] = G::lds(I.diag, x + Lx * row(-D));
            d[1] = G::lds(I.diag, x + Lx * row(1 - D));
        }
        T rnp_n = G::ld(cur, (x + Lx * row(2 - D)) * C + c);
        S dp_n = hd ? G::lds(I.diag, x + Lx * row(2 - D)) : (S)0;
        T pv_n = (!first && s >= 1 && s + 1 < Wn) ? G::template ld_s<NT>(prev, (x + Lx * row(1 - D)) * C + c) : zero;
        T m2[D], m1[D];   // level k at rows (its current row) - 2 and - 1, k = 1 .. D-1
#pragma unroll
        for (int k = 0; k < D; ++k) {
            m2[k] = zero;
            m1[k] = zero;
        }
        const uint32_t iters = ns + 2 * (D - 1);
        for (uint32_t j = 0; j < iters; ++j) {
            const T rnp = rnp_n;
            const T pv = pv_n;
            d[0] = dp_n;
            if (j + 1 < iters) {   // rows the next iteration needs
                rnp_n = G::ld(cur, (x + Lx * row((int32_t)j + 3 - D)) * C + c);
                dp_n = hd ? G::lds(I.diag, x + Lx * row((int32_t)j + 3 - D)) : (S)0;
                if (!first && s >= 1 && s + 1 < Wn)
                    pv_n = G::template ld_s<NT>(prev, (x + Lx * row((int32_t)j + 2 - D)) * C + c);
            }
            const uint32_t b = j & 1u, bp = b ^ 1u;
            lv_s[0][b][tid] = rn0;
            __syncthreads();
            T cur_k[D + 1];
            cur_k[0] = rnp;
#pragma unroll
            for (int k = 1; k <= D; ++k) {
                T v = zero;
                const bool ring = (k < D) ? (s >= (uint32_t)k && s + k < Wn) : own;
                if (ring && j >= 2u * (uint32_t)(k - 1)) {
                    if (k == 1) {
                        const T nb[4] = {lv_s[0][b][tid - C], lv_s[0][b][tid + C], rnm, rnp};
                        v = apply_real<S, 4>(hd, d[1], hop, rn0, nb);
                        if (!first) v = (S)2 * v - pv;
                    } else {
                        const T lo = (k == 2) ? rnm : m2[k - 2 > 0 ? k - 2 : 0];
                        const T nb[4] = {lv_s[k - 1][bp][tid - C], lv_s[k - 1][bp][tid + C], m2[k - 1], cur_k[k - 1]};
                        v = apply_real<S, 4>(hd, d[k], hop, m1[k - 1], nb);
                        v = (S)2 * v - lo;
                    }
                }
                cur_k[k] = v;
                // stores and dots on the owned rows [y0, y1): level k is at row offset j - D - k + 2
                const int32_t ro = (int32_t)j - D - k + 2;
                if (own && ro >= 0 && ro < (int32_t)ns) {
                    if (k == D - 1) G::template st_s<NT>(outa, (x + Lx * row(ro)) * C + c, v);
                    if (k == D) G::template st_s<NT>(outb, (x + Lx * row(ro)) * C + c, v);
                    acc[k - 1].add(v, k == 1 ? rn0 : m1[k - 1]);
                }
                if (k < D) lv_s[k][b][tid] = v;
            }
#pragma unroll
            for (int k = 1; k < D; ++k) {
                m2[k] = m1[k];
                m1[k] = cur_k[k];
            }
            rnm = rn0;
            rn0 = rnp;
#pragma unroll
            for (int q = D + 1; q > 0; --q) d[q] = d[q - 1];
        }
#pragma unroll
        for (int k = 0; k < D; ++k)
            block_reduce_store<Dots<S>::DD, TB_BLOCK>(acc[k].s0, acc[k].c0, acc[k].s1, acc[k].c1,
                                                      I.partial + (size_t)((n + 1 + k) % I.pslots) * I.tiles * 4 +
                                                          (size_t)t * 4);
    }
}

}  // namespace kpm
