// Temporal blocking of the recursion on 2D lattices with real hopping: two
// steps per pass over the vectors.
//
// One pass reads r_{n-1} and r_n and writes r_{n+1} and r_{n+2}, 4 vector
// transfers for 2 steps instead of 6.  A work item is an x-tile of T sites
// times a segment of rows (the march axis y).  Its block holds a window of
// W = TB_BLOCK / C sites (T = W - 2h owned plus h halo sites on each side;
// h = 2, or 3 when the solve also takes three-step passes, k_step_tb3), one
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

// Three steps per pass (solves whose x-tiles carry a 3-site halo): reads
// r_{n-1} and r_n and writes only r_{n+2} and r_{n+3}, which are all the next
// pass needs; r_{n+1} stays on chip (its dots are formed).  4 vector transfers
// for 3 steps.  Iteration j of an item handles row y = y0 - 2 + j of r_{n+1}
// (window minus its outer sites), row y - 1 of r_{n+2} (minus two outer sites
// each side) and row y - 2 of r_{n+3} (owned sites); in-row neighbours of all
// three come through LDS, rows y-1 .. y+1 of r_n, y-2 .. y of r_{n+1} and
// y-3 .. y-1 of r_{n+2} sit in registers.  Every value is formed with the
// one-step kernel's expression, so the vectors are bitwise those of one-step
// passes.
template <typename S, bool WIDE, bool NT>
__global__ __launch_bounds__(TB_BLOCK) void k_step_tb3(const Inst *__restrict__ tab, int32_t n, const void *prev,
                                                       const void *cur, void *out2, void *out3)
{
    typedef typename V16<S>::T T;
    typedef Mem<S, WIDE> G;
    __shared__ T rn_s[TB_BLOCK];
    __shared__ T r1_s[2][TB_BLOCK];
    __shared__ T r2_s[2][TB_BLOCK];
    const Inst I = tab[0];
    const uint32_t C = I.C, Lx = I.P, Ly = I.Lm;
    const uint32_t Wn = TB_BLOCK / C, Tn = Wn - 6;
    const uint32_t tid = threadIdx.x, s = tid / C, c = tid - s * C;
    const bool hd = I.has_diag;
    const S hop = G::lds(I.hop, 0);
    const bool first = (n == 0);
    const T zero = (T)(S)0;
    double *part1 = I.partial + (size_t)((n + 1) % I.pslots) * I.tiles * 4;
    double *part2 = I.partial + (size_t)((n + 2) % I.pslots) * I.tiles * 4;
    double *part3 = I.partial + (size_t)((n + 3) % I.pslots) * I.tiles * 4;
    const ItemRange ir = item_range(I, I.nct, I.nseg);
    for (uint32_t it = ir.first; it < ir.count; it += ir.stride) {
        const uint32_t sl = it / ir.nu;
        const uint32_t sg = ir.sb + sl;
        const uint32_t tx = ir.ub + (it - sl * ir.nu);
        const uint32_t x0 = tx * Tn;
        const uint32_t xend = min(x0 + Tn, Lx);
        const uint32_t x = (x0 + Lx - 3 + s) % Lx;
        const bool own = s >= 3 && s < Wn - 3 && x0 + s - 3 < xend;
        const bool ring1 = s >= 1 && s + 1 < Wn;
        const bool ring2 = s >= 2 && s + 2 < Wn;
        const uint32_t y0 = sg * I.S, y1 = min(y0 + I.S, Ly), ns = y1 - y0;
        const uint32_t t = sg * I.nct + tx;
        Dots<S> a1, a2, a3;
        auto row = [&](int32_t off) { return (y0 + Ly + (uint32_t)off) % Ly; };   // y0 + off, periodic
        T rnm = G::ld(cur, (x + Lx * row(-3)) * C + c);
        T rn0 = G::ld(cur, (x + Lx * row(-2)) * C + c);
        S dm2 = (S)0;
        S dm = hd ? G::lds(I.diag, x + Lx * row(-3)) : (S)0;
        S d0 = hd ? G::lds(I.diag, x + Lx * row(-2)) : (S)0;
        // row y0-1 of r_n (and its diagonal) and row y0-2 of r_{n-1}, one row ahead
        T rnp_n = G::ld(cur, (x + Lx * row(-1)) * C + c);
        S dp_n = hd ? G::lds(I.diag, x + Lx * row(-1)) : (S)0;
        T pv_n = (ring1 && !first) ? G::template ld_s<NT>(prev, (x + Lx * row(-2)) * C + c) : zero;
        T r1m2 = zero, r1m1 = zero, r2m2 = zero, r2m1 = zero;
        for (uint32_t j = 0; j <= ns + 3; ++j) {
            const T rnp = rnp_n;
            const S dp = dp_n;
            const T pv = pv_n;
            if (j <= ns + 2) {   // rows the next iteration needs
                rnp_n = G::ld(cur, (x + Lx * row((int32_t)j)) * C + c);
                dp_n = hd ? G::lds(I.diag, x + Lx * row((int32_t)j)) : (S)0;
                if (ring1 && !first) pv_n = G::template ld_s<NT>(prev, (x + Lx * row((int32_t)j - 1)) * C + c);
            }
            // r_{n+1}, row y
            rn_s[tid] = rn0;
            __syncthreads();
            T r1 = zero;
            if (ring1) {
                const T nb[4] = {rn_s[tid - C], rn_s[tid + C], rnm, rnp};
                r1 = apply_real<S, 4>(hd, d0, hop, rn0, nb);
                if (!first) r1 = (S)2 * r1 - pv;
            }
            if (own && j >= 2 && j <= ns + 1) a1.add(r1, rn0);
            r1_s[j & 1][tid] = r1;
            __syncthreads();
            // r_{n+2}, row y - 1
            T r2 = zero;
            if (j >= 2 && ring2) {
                const T nb[4] = {r1_s[(j - 1) & 1][tid - C], r1_s[(j - 1) & 1][tid + C], r1m2, r1};
                r2 = apply_real<S, 4>(hd, dm, hop, r1m1, nb);
                r2 = (S)2 * r2 - rnm;
            }
            if (own && j >= 3 && j <= ns + 2) {
                G::template st_s<NT>(out2, (x + Lx * row((int32_t)j - 3)) * C + c, r2);
                a2.add(r2, r1m1);
            }
            r2_s[j & 1][tid] = r2;
            __syncthreads();
            // r_{n+3}, row y - 2
            if (own && j >= 4) {
                const T nb[4] = {r2_s[(j - 1) & 1][tid - C], r2_s[(j - 1) & 1][tid + C], r2m2, r2};
                T r3 = apply_real<S, 4>(hd, dm2, hop, r2m1, nb);
                r3 = (S)2 * r3 - r1m2;
                G::template st_s<NT>(out3, (x + Lx * row((int32_t)j - 4)) * C + c, r3);
                a3.add(r3, r2m1);
            }
            r2m2 = r2m1;
            r2m1 = r2;
            r1m2 = r1m1;
            r1m1 = r1;
            rnm = rn0;
            rn0 = rnp;
            dm2 = dm;
            dm = d0;
            d0 = dp;
        }
        block_reduce_store<Dots<S>::DD, TB_BLOCK>(a1.s0, a1.c0, a1.s1, a1.c1, part1 + (size_t)t * 4);
        block_reduce_store<Dots<S>::DD, TB_BLOCK>(a2.s0, a2.c0, a2.s1, a2.c1, part2 + (size_t)t * 4);
        block_reduce_store<Dots<S>::DD, TB_BLOCK>(a3.s0, a3.c0, a3.s1, a3.c1, part3 + (size_t)t * 4);
    }
}

}  // namespace kpm
