// Temporal blocking of the recursion on 3D lattices (real or spin hopping):
// two steps per pass over the vectors.
//
// Layout.  A solve run by these kernels stores its vectors chunk-major: chunk
// c of site i at 16-byte index c N + i, so that a block working on one chunk
// of a whole plane reads and writes contiguous memory.  (The other kernels
// keep the site-major layout; only these kernels touch this solve's vectors.)
//
// Work item: one chunk c x one row tile of a plane x one segment of planes
// along z.  A row tile owns rows [y0, y0 + T) of every plane and also holds
// two rows of r_n on each side (none when one tile spans the whole plane,
// whose rows then wrap inside the tile), every x; its elements (rows x L_x, at
// most TB3_TILE) are spread over the block's threads, TB3_EPT per thread.
// The block marches the segment's planes in z, keeping for each element r_n
// at planes z - 1, z, z + 1 and level 1 (r_{n+1}) at z - 2, z - 1 in registers.
// At plane z it copies r_n into LDS, forms level 1 on all but the outermost
// rows (in-plane neighbours from the LDS copy of r_n), copies it into LDS, and
// forms level 2 (r_{n+2}) at plane z - 1 on the owned rows (in-plane
// neighbours from the LDS copy of level 1 at z - 1).  Both LDS planes
// alternate between two buffers, so one block barrier per plane suffices, and
// the next plane's r_n, r_{n-1} and diagonal are loaded a plane ahead.  A
// segment [z0, z1) forms level 1 on planes z0 - 1 .. z1 (reading r_n on
// z0 - 2 .. z1 + 1, r_{n-1} on z0 - 1 .. z1) and level 2 on z0 .. z1 - 1.
// Every value is formed with the one-step kernels' expression in their slot
// order, so the vectors are bitwise those of one-step passes.
//
// A pass reads r_{n-1}, r_n and writes r_{n+1} (outa) and r_{n+2} (outb): with
// the halo rows and planes about 4.5 to 5 vector streams for two steps where
// the one-step kernels move 6.5.  A single step (D = 1) writes r_{n+1} to outb.
#pragma once

namespace kpm {

constexpr int TB3_BLOCK = 512;
constexpr int TB3_EPT = 2;                                  // tile elements per thread
constexpr uint32_t TB3_TILE = (uint32_t)TB3_BLOCK * TB3_EPT;  // elements (sites x one chunk) per tile
constexpr int MODE_TB3 = 4;                                 // plan mode of solves run by these kernels

// Geometry of one work item of a 3D blocked solve (Inst: P = owned rows per
// tile T, nct = row tiles per plane, Lm = L_z, S = planes per segment).
struct Tb3Item {
    uint32_t c, y0, rows, hy, et, z0, z1;
    bool whole;   // one tile spans the plane: no halo rows, rows wrap inside the tile
};
__device__ __forceinline__ Tb3Item tb3_item(const Inst &I, uint32_t unit, uint32_t sg)
{
    Tb3Item t;
    const uint32_t ty = unit / I.C;
    t.c = unit - ty * I.C;
    t.whole = (I.nct == 1);
    t.y0 = ty * I.P;
    t.rows = min(I.P, I.Ly - t.y0);
    t.hy = t.whole ? I.Ly : t.rows + 4;
    t.et = t.hy * I.Lx;
    t.z0 = sg * I.S;
    t.z1 = min(t.z0 + I.S, I.Lz);
    return t;
}

// Per-element geometry inside a tile: in-plane site, its neighbours -x, +x, -y,
// +y as tile elements (for the LDS planes), and which levels it forms.
struct Tb3Elem {
    uint32_t p, pxm, pym;   // in-plane site and its -x, -y neighbours (their forward bonds)
    uint32_t q, qx[4];      // tile element (its LDS slot) and those of -x, +x, -y, +y
    bool valid, lv1, own;   // in the tile; forms level 1; owned (forms level 2, stores)
};
__device__ __forceinline__ Tb3Elem tb3_elem(const Inst &I, const Tb3Item &t, uint32_t q)
{
    Tb3Elem e;
    const uint32_t Lx = I.Lx, Ly = I.Ly;
    e.valid = q < t.et;
    // elements beyond the tile take site 0 of it for their (unused) loads and keep their own,
    // otherwise unused, LDS slot q < TB3_TILE
    const uint32_t qq = e.valid ? q : 0u;
    e.q = q;
    const uint32_t r = fdiv(qq, I.fLx);
    const uint32_t x = qq - r * Lx;
    const uint32_t y = t.whole ? r : (t.y0 + Ly - 2 + r) % Ly;
    e.lv1 = e.valid && (t.whole || (r >= 1 && r + 1 < t.hy));
    e.own = e.valid && (t.whole || (r >= 2 && r + 2 < t.hy));
    e.p = x + Lx * y;
    e.pxm = (x == 0) ? e.p + (Lx - 1) : e.p - 1;
    e.pym = (y == 0) ? e.p + (Ly - 1) * Lx : e.p - Lx;
    e.qx[0] = (x == 0) ? qq + (Lx - 1) : qq - 1;
    e.qx[1] = (x == Lx - 1) ? qq - (Lx - 1) : qq + 1;
    if (t.whole) {
        e.qx[2] = (r == 0) ? qq + (Ly - 1) * Lx : qq - Lx;
        e.qx[3] = (r == Ly - 1) ? qq - (Ly - 1) * Lx : qq + Lx;
    } else {   // only rows 1 .. hy - 2 read these; the outermost get a harmless in-tile index
        e.qx[2] = (r >= 1) ? qq - Lx : qq;
        e.qx[3] = (r + 1 < t.hy) ? qq + Lx : qq;
    }
    return e;
}

// r_0 in the chunk-major layout (and the partials of <r_0|r_0>, slot 0) over the
// solve's work items (owned rows and planes of each).
template <typename S, bool WIDE>
__global__ __launch_bounds__(TB3_BLOCK) void k_init_tb3(const Inst *__restrict__ tab, void *cur)
{
    typedef Mem<S, WIDE> G;
    const Inst I = tab[0];
    const uint32_t N = I.N, P = I.Lx * I.Ly;
    const ItemRange ir = item_range(I, I.C * I.nct, I.nseg);
    for (uint32_t it = ir.first; it < ir.count; it += ir.stride) {
        const uint32_t sl = it / ir.nu;
        const uint32_t sg = ir.sb + sl;
        const uint32_t unit = ir.ub + (it - sl * ir.nu);
        const Tb3Item t = tb3_item(I, unit, sg);
        Dots<S> a;
#pragma unroll
        for (int u = 0; u < TB3_EPT; ++u) {
            const Tb3Elem e = tb3_elem(I, t, threadIdx.x + (uint32_t)u * TB3_BLOCK);
            if (!e.own) continue;
            for (uint32_t z = t.z0; z < t.z1; ++z) {
                const uint32_t i = e.p + P * z;
                const auto v = start_chunk<S>(I, i, t.c);
                G::st(cur, t.c * N + i, v);
                a.norm_only(v);
            }
        }
        block_reduce_store<Dots<S>::DD, TB3_BLOCK>(a.s0, a.c0, a.s1, a.c1, I.partial + (size_t)(sg * I.nct * I.C + unit) * 4);
    }
}

// One or two recursion steps (D) per launch on a 3D lattice, chunk-major vectors.
// Solo launches (bmap == nullptr): tab[0] at step n = arg with the buffers given;
// batched launches: the block map's instances run one pass of their chunk
// (tb_pass_roles).
template <typename S, int OPK, bool WIDE, bool NT, int D>
__global__ __launch_bounds__(TB3_BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_step_tb3(
    const Inst *__restrict__ tab, const uint32_t *__restrict__ bmap, int32_t arg, const void *prev, const void *cur,
    void *outa, void *outb)
{
    typedef typename V16<S>::T T;
    typedef Mem<S, WIDE> G;
    typedef typename Mem<S, WIDE>::S2 S2;
    constexpr bool SPIN = (OPK == OP_SPIN3);
    constexpr int NS = 6;
    __shared__ T lr[2][TB3_TILE];                              // r_n at plane z
    __shared__ T lv[D == 2 ? 2 : 1][D == 2 ? TB3_TILE : 1];    // level 1 at plane z
    const uint32_t hb = bmap ? bmap[blockIdx.x] : 0u;
    if (hb == NO_INSTANCE) return;
    const Inst I = tab[hb];
    int32_t n = arg;
    if (bmap && !tb_pass_roles(I, arg, D, n, prev, cur, outa, outb)) return;
    const uint32_t N = I.N, Lz = I.Lz, P = I.Lx * I.Ly;
    const bool first = (n == 0);
    const bool hd = I.has_diag;
    const S hop = SPIN ? (S)0 : G::lds(I.hop, 0);
    const T zero = (T)(S)0;
    const ItemRange ir = item_range(I, I.C * I.nct, I.nseg);
    for (uint32_t it = ir.first; it < ir.count; it += ir.stride) {
        const uint32_t sl = it / ir.nu;
        const uint32_t sg = ir.sb + sl;
        const uint32_t unit = ir.ub + (it - sl * ir.nu);
        const Tb3Item t = tb3_item(I, unit, sg);
        const uint32_t cb = t.c * N;   // this chunk's plane of the vectors
        Tb3Elem e[TB3_EPT];
#pragma unroll
        for (int u = 0; u < TB3_EPT; ++u) e[u] = tb3_elem(I, t, threadIdx.x + (uint32_t)u * TB3_BLOCK);
        Dots<S> acc1, acc2;
        // level 1 runs on planes z0 - 1 .. z1 for two steps, z0 .. z1 - 1 for one
        const uint32_t ns = t.z1 - t.z0;
        const uint32_t iters = (D == 2) ? ns + 2 : ns;
        uint32_t zc = (D == 2) ? (t.z0 + Lz - 1) % Lz : t.z0;          // plane of level 1
        uint32_t zm = (zc + Lz - 1) % Lz, zp = (zc + 1 == Lz) ? 0 : zc + 1;
        T rm[TB3_EPT], r0[TB3_EPT], rp[TB3_EPT];   // r_n at planes zc - 1, zc, zc + 1
        T va[TB3_EPT], vb[TB3_EPT];                // level 1 at planes zc - 2, zc - 1
        T pv[TB3_EPT];                             // r_{n-1} at plane zc
        S d0[TB3_EPT], dm[TB3_EPT];                // diagonal at planes zc, zc - 1
#pragma unroll
        for (int u = 0; u < TB3_EPT; ++u) {
            const uint32_t p = e[u].p;
            rm[u] = G::ld(cur, cb + p + P * zm);
            r0[u] = G::ld(cur, cb + p + P * zc);
            rp[u] = G::ld(cur, cb + p + P * zp);
            pv[u] = (!first && e[u].lv1) ? G::template ld_s<NT>(prev, cb + p + P * zc) : zero;
            d0[u] = hd ? G::lds(I.diag, p + P * zc) : (S)0;
            va[u] = zero;
            vb[u] = zero;
            dm[u] = (S)0;
            lr[0][e[u].q] = r0[u];
        }
        __syncthreads();
        for (uint32_t j = 0; j < iters; ++j) {
            const uint32_t zn = (zp + 1 == Lz) ? 0 : zp + 1;   // plane zc + 2
            const uint32_t b = j & 1u;
            const bool own_z1 = (D == 1) || (j >= 1 && j <= ns);   // level 1's plane zc is owned
            T v1[TB3_EPT];
#pragma unroll
            for (int u = 0; u < TB3_EPT; ++u) {
                const Tb3Elem &E = e[u];
                const uint32_t i = E.p + P * zc;
                T nb[NS];
                nb[0] = lr[b][E.qx[0]];
                nb[1] = lr[b][E.qx[1]];
                nb[2] = lr[b][E.qx[2]];
                nb[3] = lr[b][E.qx[3]];
                nb[4] = rm[u];
                nb[5] = rp[u];
                T out;
                if (!SPIN) {
                    out = apply_real<S, NS>(hd, d0[u], hop, r0[u], nb);
                } else {
                    // forward bonds of the site and of its -x, -y, -z neighbours (the backward
                    // bonds are their conjugates)
                    S hr[NS], hi[NS];
                    const S2 bxm = G::ldc(I.bond, (E.pxm + P * zc) * 3 + 0);
                    const S2 bxp = G::ldc(I.bond, i * 3 + 0);
                    const S2 bym = G::ldc(I.bond, (E.pym + P * zc) * 3 + 1);
                    const S2 byp = G::ldc(I.bond, i * 3 + 1);
                    const S2 bzm = G::ldc(I.bond, (E.p + P * zm) * 3 + 2);
                    const S2 bzp = G::ldc(I.bond, i * 3 + 2);
                    hr[0] = bxm[0]; hi[0] = -bxm[1];
                    hr[1] = bxp[0]; hi[1] = bxp[1];
                    hr[2] = bym[0]; hi[2] = -bym[1];
                    hr[3] = byp[0]; hi[3] = byp[1];
                    hr[4] = bzm[0]; hi[4] = -bzm[1];
                    hr[5] = bzp[0]; hi[5] = bzp[1];
                    out = apply_cplx<S, NS>(hd, d0[u], r0[u], nb, hr, hi);
                }
                if (!first) out = (S)2 * out - pv[u];
                v1[u] = out;
                if (E.own && own_z1) {
                    G::template st_s<NT>(D == 2 ? outa : outb, cb + i, out);
                    acc1.add(out, r0[u]);
                }
                if constexpr (D == 2) lv[b][E.q] = out;
            }
            if constexpr (D == 2) {
                // level 2 at plane zc - 1 on the owned rows, for planes z0 .. z1 - 1
                if (j >= 2) {
#pragma unroll
                    for (int u = 0; u < TB3_EPT; ++u) {
                        const Tb3Elem &E = e[u];
                        if (!E.own) continue;
                        const uint32_t i = E.p + P * zm;
                        const uint32_t bpv = b ^ 1u;
                        T nb[NS];
                        nb[0] = lv[bpv][E.qx[0]];
                        nb[1] = lv[bpv][E.qx[1]];
                        nb[2] = lv[bpv][E.qx[2]];
                        nb[3] = lv[bpv][E.qx[3]];
                        nb[4] = va[u];
                        nb[5] = v1[u];
                        T out;
                        if (!SPIN) {
                            out = apply_real<S, NS>(hd, dm[u], hop, vb[u], nb);
                        } else {
                            const uint32_t zmm = (zm + Lz - 1) % Lz;
                            S hr[NS], hi[NS];
                            const S2 bxm = G::ldc(I.bond, (E.pxm + P * zm) * 3 + 0);
                            const S2 bxp = G::ldc(I.bond, i * 3 + 0);
                            const S2 bym = G::ldc(I.bond, (E.pym + P * zm) * 3 + 1);
                            const S2 byp = G::ldc(I.bond, i * 3 + 1);
                            const S2 bzm = G::ldc(I.bond, (E.p + P * zmm) * 3 + 2);
                            const S2 bzp = G::ldc(I.bond, i * 3 + 2);
                            hr[0] = bxm[0]; hi[0] = -bxm[1];
                            hr[1] = bxp[0]; hi[1] = bxp[1];
                            hr[2] = bym[0]; hi[2] = -bym[1];
                            hr[3] = byp[0]; hi[3] = byp[1];
                            hr[4] = bzm[0]; hi[4] = -bzm[1];
                            hr[5] = bzp[0]; hi[5] = bzp[1];
                            out = apply_cplx<S, NS>(hd, dm[u], vb[u], nb, hr, hi);
                        }
                        out = (S)2 * out - rm[u];
                        G::template st_s<NT>(outb, cb + i, out);
                        acc2.add(out, vb[u]);
                    }
                }
            }
            // advance one plane: r_n at zc + 1 into the other LDS buffer, the next plane's
            // loads issued now
            if (j + 1 < iters) {
#pragma unroll
                for (int u = 0; u < TB3_EPT; ++u) {
                    const uint32_t p = e[u].p;
                    lr[b ^ 1u][e[u].q] = rp[u];
                    va[u] = vb[u];
                    vb[u] = v1[u];
                    dm[u] = d0[u];
                    rm[u] = r0[u];
                    r0[u] = rp[u];
                    rp[u] = G::ld(cur, cb + p + P * zn);
                    pv[u] = (!first && e[u].lv1) ? G::template ld_s<NT>(prev, cb + p + P * zp) : zero;
                    d0[u] = hd ? G::lds(I.diag, p + P * zp) : (S)0;
                }
                zm = zc;
                zc = zp;
                zp = zn;
            }
            __syncthreads();
        }
        const uint32_t tslot = sg * I.nct * I.C + unit;
        block_reduce_store<Dots<S>::DD, TB3_BLOCK>(acc1.s0, acc1.c0, acc1.s1, acc1.c1,
                                                   I.partial + (size_t)((n + 1) % I.pslots) * I.tiles * 4 +
                                                       (size_t)tslot * 4);
        if constexpr (D == 2)
            block_reduce_store<Dots<S>::DD, TB3_BLOCK>(acc2.s0, acc2.c0, acc2.s1, acc2.c1,
                                                       I.partial + (size_t)((n + 2) % I.pslots) * I.tiles * 4 +
                                                           (size_t)tslot * 4);
    }
}

}  // namespace kpm
