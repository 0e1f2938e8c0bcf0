// Temporal blocking of the recursion on 2D lattices (real or spin hopping):
// several steps per pass over the vectors.
//
// A work item is an x-tile of T sites times a segment of rows (the march axis
// y) times one group of the site's chunks (C / G of its C 16-byte chunks, G
// groups; smaller groups widen the window and so cut the halo's share).  Its
// block holds a window of W = TB_BLOCK / (C / G) sites (T = W - 2h owned plus
// h halo sites on each side, h = the depth of the solve's deepest passes), one
// thread per 16-byte chunk of the group.  A pass of D <= h steps reads r_{n-1} and r_n
// and writes r_{n+D-1} and r_{n+D} (for D = 1 only r_{n+1}); the halo
// recomputation means r_{n-1} and r_n are read by neighbouring tiles while the
// pass runs, so the outputs go to the two free buffers of four.  r_{n-1} (read
// once) and the outputs (written once) use non-temporal accesses when the
// instance streams.
#pragma once

namespace kpm {

constexpr int TB_BLOCK = 512;
constexpr int MODE_TB = 3;   // plan mode of solves run by these kernels
// Passes shallow enough for two blocks per CU in LDS (D <= 4: 16 KiB per level)
// are held to 128 VGPRs (4 waves per SIMD), so that the second block fits.
#define TB_WAVES_PER_EU(S, D) ((sizeof(S) == 4 ? (D) <= 4 : (D) <= 3) ? 4 : 1)

// Batched passes: the pass a launch with argument `arg` runs for instance I
// (arg >= 0: full-depth pass arg of the chunk, D = tbh; arg < 0: the remainder
// pass, D = tbrem), its first step n and its buffer roles.  Pass j starts at
// step step0 + j * tbh; a pass of depth >= 2 writes its two outputs to the two
// buffers not holding (r_{n-1}, r_n), in ascending order, so pass j reads the
// chunk's starting pair (tbp, tbc) itself (j = 0), its complement (j odd) or
// the pair in ascending order (j even >= 2).  False if I has no such pass.
__device__ __forceinline__ bool tb_pass_roles(const Inst &I, int32_t arg, int D, int32_t &n, const void *&prev,
                                              const void *&cur, void *&outa, void *&outb)
{
    int32_t j = arg;
    if (arg < 0) {
        if (I.tbrem != D) return false;
        j = I.tbfull;
    } else if (j >= I.tbfull) {
        return false;
    }
    n = I.step0 + j * I.tbh;
    void *const bufs[4] = {I.buf0, I.buf1, I.tb2, I.tb3};
    int p = I.tbp, c = I.tbc;
    if (j > 0) {
        const int lo = min(p, c), hi = max(p, c);
        int f0 = 0;
        while (f0 == lo || f0 == hi) ++f0;
        int f1 = f0 + 1;
        while (f1 == lo || f1 == hi) ++f1;
        p = (j & 1) ? f0 : lo;
        c = (j & 1) ? f1 : hi;
    }
    int f0 = 0;
    while (f0 == p || f0 == c) ++f0;
    int f1 = f0 + 1;
    while (f1 == p || f1 == c) ++f1;
    prev = bufs[p];
    cur = bufs[c];
    outa = bufs[D >= 2 ? f0 : f1];
    outb = bufs[D >= 2 ? f1 : f0];
    return true;
}

// r_0 (and the partials of <r_0|r_0>, slot 0) into `cur` over the solve's work
// items (the owned sites of each tile and segment).
template <typename S, bool WIDE>
__global__ __launch_bounds__(TB_BLOCK) void k_init_tb(const Inst *__restrict__ tab, void *cur)
{
    typedef typename V16<S>::T T;
    typedef Mem<S, WIDE> G;
    const Inst I = tab[0];
    const uint32_t C = I.C, Gs = I.tbg, Cg = C / Gs, Lx = I.P, Ly = I.Lm;
    const uint32_t h = (uint32_t)I.tbh, Wn = TB_BLOCK / Cg, Tn = Wn - 2 * h;
    const uint32_t tid = threadIdx.x, s = tid / Cg, cl = tid - s * Cg;
    const ItemRange ir = item_range(I, I.nct * Gs, I.nseg);
    for (uint32_t it = ir.first; it < ir.count; it += ir.stride) {
        const uint32_t sl = it / ir.nu;
        const uint32_t sg = ir.sb + sl;
        const uint32_t unit = ir.ub + (it - sl * ir.nu);
        const uint32_t tx = unit / Gs, c = (unit - tx * Gs) * Cg + cl;
        const uint32_t x0 = tx * Tn;
        const uint32_t xend = min(x0 + Tn, Lx);
        const uint32_t x = (x0 + Lx - h + s) % Lx;
        const bool own = s >= h && s < Wn - h && x0 + s - h < xend;
        const uint32_t y0 = sg * I.S, y1 = min(y0 + I.S, Ly);
        Dots<S> a;
        if (own)
            for (uint32_t y = y0; y < y1; ++y) {
                const uint32_t i = x + Lx * y;
                const T v = start_chunk<S>(I, i, c);
                G::st(cur, i * C + c, v);
                a.norm_only(v);
            }
        block_reduce_store<Dots<S>::DD, TB_BLOCK>(a.s0, a.c0, a.s1, a.c1,
                                                  I.partial + (size_t)(sg * I.nct * Gs + unit) * 4);
    }
}

// Depth-D passes (D = 1 .. 6, D <= the tiles' halo h): one launch advances D
// steps.  It reads r_{n-1} and r_n and writes only r_{n+D-1} and r_{n+D}, all
// the next pass needs; r_{n+1} .. r_{n+D-2} exist only on chip, where their
// dots are formed: 4 vector transfers for D steps (a single step writes r_{n+1}
// to `outb` only).  Level k = 1..D computes r_{n+k}; at iteration j (row
// y = y0 - (D-1) + j) level k handles row y - (k-1) on the sites at least k
// from the window edge (level D: the owned sites), from level k-1 at rows
// y - k .. y - k + 2 (level 0 = r_n, rows y - 1 .. y + 1) and level k-2 at
// row y - (k-1) (r_{n-1} for level 1).  In-row neighbours come through LDS,
// every level's row double-buffered so that one block barrier per row
// suffices; rows in registers otherwise.  Every value is formed with the
// one-step kernel's expression, so the vectors are bitwise those of one-step
// passes.
//
// Solo launches (bmap == nullptr) take the instance tab[0], the step n = arg and
// the four buffer roles from the arguments.  Batched launches take the instance
// from the block map and run one pass of its current chunk (tb_pass_roles).
template <typename S, int OPK, bool WIDE, bool NT, int D>
__global__ __launch_bounds__(TB_BLOCK) __attribute__((amdgpu_waves_per_eu(TB_WAVES_PER_EU(S, D)))) void k_step_tbd(
    const Inst *__restrict__ tab, const uint32_t *__restrict__ bmap, int32_t arg, const void *prev, const void *cur,
    void *outa, void *outb)
{
    typedef typename V16<S>::T T;
    typedef Mem<S, WIDE> G;
    typedef typename Mem<S, WIDE>::S2 S2;
    constexpr bool SPIN = (OPK == OP_SPIN2);
    __shared__ T lv_s[D][2][TB_BLOCK];   // level k's row of the iteration, double-buffered (k < D)
    const uint32_t hb = bmap ? bmap[blockIdx.x] : 0u;
    if (hb == NO_INSTANCE) return;
    const Inst I = tab[hb];
    int32_t n = arg;
    if (bmap && !tb_pass_roles(I, arg, D, n, prev, cur, outa, outb)) return;
    const uint32_t C = I.C, Gs = I.tbg, Cg = C / Gs, Lx = I.P, Ly = I.Lm;
    const uint32_t h = (uint32_t)I.tbh, Wn = TB_BLOCK / Cg, Tn = Wn - 2 * h;   // h >= D
    const uint32_t tid = threadIdx.x, s = tid / Cg, cl = tid - s * Cg;
    const bool hd = I.has_diag;
    const S hop = SPIN ? (S)0 : G::lds(I.hop, 0);
    const bool first = (n == 0);
    const T zero = (T)(S)0;
    const T two = (T)(S)2;
    const ItemRange ir = item_range(I, I.nct * Gs, I.nseg);
    for (uint32_t it = ir.first; it < ir.count; it += ir.stride) {
        const uint32_t sl = it / ir.nu;
        const uint32_t sg = ir.sb + sl;
        const uint32_t unit = ir.ub + (it - sl * ir.nu);
        const uint32_t tx = unit / Gs, c = (unit - tx * Gs) * Cg + cl;
        const uint32_t x0 = tx * Tn;
        const uint32_t xend = min(x0 + Tn, Lx);
        const uint32_t x = (x0 + Lx - h + s) % Lx;
        const uint32_t xm = (x == 0) ? Lx - 1 : x - 1;   // -x neighbour (its forward x-bond)
        const bool own = s >= h && s < Wn - h && x0 + s - h < xend;
        const uint32_t y0 = sg * I.S, y1 = min(y0 + I.S, Ly), ns = y1 - y0;
        const uint32_t t = sg * I.nct * Gs + unit;
        const uint32_t tl = (s >= 1) ? tid - Cg : tid, tr = (s + 1 < Wn) ? tid + Cg : tid;   // in-row neighbours
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
        // rows advance by one per iteration, tracked without divisions: yc = y0 + j + 2 - D (periodic)
        uint32_t yc = row(2 - D);
        T rnp_n = G::ld(cur, (x + Lx * yc) * C + c);
        S dp_n = hd ? G::lds(I.diag, x + Lx * yc) : (S)0;
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
                const uint32_t yn = (yc + 1 == Ly) ? 0 : yc + 1;
                rnp_n = G::ld(cur, (x + Lx * yn) * C + c);
                dp_n = hd ? G::lds(I.diag, x + Lx * yn) : (S)0;
                if (!first && s >= 1 && s + 1 < Wn)
                    pv_n = G::template ld_s<NT>(prev, (x + Lx * yc) * C + c);
            }
            const uint32_t b = j & 1u, bp = b ^ 1u;
            lv_s[0][b][tid] = rn0;
            __syncthreads();
            T cur_k[D + 1];
            cur_k[0] = rnp;
#pragma unroll
            for (int k = 1; k <= D; ++k) {
                // level k's row y - (k-1) on every site of the window: the levels above read only
                // the sites at least k from the window edge, and only once the pipeline has filled
                // (j >= 2(k-1)), so the values elsewhere are never used (edge neighbours are
                // clamped to the site itself to keep the reads in the row)
                // centre, neighbours (slots -x, +x, -y, +y), value subtracted (r_{n+k-2} at that row)
                T centre, sub;
                T nb[4];
                if (k == 1) {
                    centre = rn0;
                    nb[0] = lv_s[0][b][tl];
                    nb[1] = lv_s[0][b][tr];
                    nb[2] = rnm;
                    nb[3] = rnp;
                    sub = pv;
                } else {
                    centre = m1[k - 1];
                    nb[0] = lv_s[k - 1][bp][tl];
                    nb[1] = lv_s[k - 1][bp][tr];
                    nb[2] = m2[k - 1];
                    nb[3] = cur_k[k - 1];
                    sub = (k == 2) ? rnm : m2[k - 2 > 0 ? k - 2 : 0];
                }
                T v;
                if constexpr (SPIN) {
                    // bonds H~_{i,i+x}, H~_{i,i+y} stored at site i; the backward ones are the
                    // conjugates of the neighbour's forward bonds
                    // rows yc - k and yc - k - 1; k + 1 <= D <= L_y / 2, so one wrap at most
                    const uint32_t ry = (yc >= (uint32_t)k) ? yc - k : yc + Ly - k;
                    const uint32_t rym = (ry == 0) ? Ly - 1 : ry - 1;
                    const S2 bxm = G::ldc(I.bond, (xm + Lx * ry) * 2 + 0);
                    const S2 bxp = G::ldc(I.bond, (x + Lx * ry) * 2 + 0);
                    const S2 bym = G::ldc(I.bond, (x + Lx * rym) * 2 + 1);
                    const S2 byp = G::ldc(I.bond, (x + Lx * ry) * 2 + 1);
                    const S hr[4] = {bxm[0], bxp[0], bym[0], byp[0]};
                    const S hi[4] = {-bxm[1], bxp[1], -bym[1], byp[1]};
                    v = apply_cplx<S, 4>(hd, d[k], centre, nb, hr, hi);
                } else {
                    v = apply_real<S, 4>(hd, d[k], hop, centre, nb);
                }
                // 2 v - sub in one rounding (2 v is exact), as the one-step kernel's expression
                if (k > 1 || !first) v = __builtin_elementwise_fma(two, v, -sub);
                cur_k[k] = v;
                // stores and dots on the owned rows [y0, y1): level k is at row offset j - D - k + 2
                const int32_t ro = (int32_t)j - D - k + 2;
                if (own && ro >= 0 && ro < (int32_t)ns) {
                    if (k == D - 1) G::template st_s<NT>(outa, (x + Lx * (y0 + ro)) * C + c, v);
                    if (k == D) G::template st_s<NT>(outb, (x + Lx * (y0 + ro)) * C + c, v);
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
            yc = (yc + 1 == Ly) ? 0 : yc + 1;
        }
#pragma unroll
        for (int k = 0; k < D; ++k)
            block_reduce_store<Dots<S>::DD, TB_BLOCK>(acc[k].s0, acc[k].c0, acc[k].s1, acc[k].c1,
                                                      I.partial + (size_t)((n + 1 + k) % I.pslots) * I.tiles * 4 +
                                                          (size_t)t * 4);
    }
}

}  // namespace kpm
