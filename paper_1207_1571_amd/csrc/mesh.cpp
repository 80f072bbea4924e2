// Mesh ingest: validation, face canonicalisation and the cell-to-face index
// ranges that every cell gather uses (host side, once per mesh).
//
// The paper's problem statement (Section 3.1) fixes what a mesh is: cells,
// faces owned by one cell and shared with at most one neighbour, geometry
// per face.  It keeps face data addressable both "by rows" and "by columns"
// through an ELL table plus a transpose-slot table (Section 3.1).  Here the
// same two access directions come from sorting: internal faces are
// canonicalised to owner < neighbour and sorted by (owner, neighbour), so a
// cell's owned faces are one contiguous range; a second index (losort) lists
// the faces ordered by (neighbour, owner), so the faces a cell sees from the
// neighbour side are a contiguous range of it.  Face coefficients are stored
// once per face and read from both sides.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "fvm_internal.h"

std::string &fvm_err_buf();
fvm_status fvm_fail(fvm_status code, const std::string &msg);

namespace {

bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// Sliced-ELL structure of the off-diagonal part (see fvm_mesh).  Slot
// order is ascending column in both slice modes, so a cell sums its entries
// in the same order whether its slice is regular or explicit.
void build_sell(fvm_mesh *m)
{
    const int32_t N = m->N;
    const int32_t ns = (N + kBlock - 1) / kBlock;
    int32_t W = 0;
    for (int32_t i = 0; i < N; ++i)
        W = std::max(W, (m->own_start[i + 1] - m->own_start[i]) + (m->nbr_start[i + 1] - m->nbr_start[i]));
    W = std::max(W, 1);
    m->sell_W = W;
    const size_t E = (size_t)ns * W * kBlock;
    m->sell_mode.assign(ns, 0);
    m->sell_off.assign((size_t)ns * W, 0);
    m->sell_fe.assign(E, -1);
    m->sell_col.assign(E, 0);
    std::vector<std::pair<int32_t, int32_t>> ent;   // (column, code) of one cell
    std::vector<int32_t> offs;
    for (int32_t s = 0; s < ns; ++s) {
        const int32_t i0 = s * kBlock, i1 = std::min(N, i0 + kBlock);
        offs.clear();
        for (int32_t i = i0; i < i1; ++i) {
            for (int32_t f = m->own_start[i]; f < m->own_start[i + 1]; ++f) offs.push_back(m->nei[f] - i);
            for (int32_t k = m->nbr_start[i]; k < m->nbr_start[i + 1]; ++k) offs.push_back(m->own[m->losort[k]] - i);
        }
        std::sort(offs.begin(), offs.end());
        offs.erase(std::unique(offs.begin(), offs.end()), offs.end());
        const bool regular = (int32_t)offs.size() <= W;
        m->sell_mode[s] = regular ? 0 : 1;
        if (regular)
            for (size_t k = 0; k < offs.size(); ++k) m->sell_off[(size_t)s * W + k] = offs[k];
        for (int32_t i = i0; i < i1; ++i) {
            ent.clear();
            for (int32_t f = m->own_start[i]; f < m->own_start[i + 1]; ++f) ent.push_back({m->nei[f], 2 * f});
            for (int32_t k = m->nbr_start[i]; k < m->nbr_start[i + 1]; ++k) {
                const int32_t f = m->losort[k];
                ent.push_back({m->own[f], 2 * f + 1});
            }
            std::sort(ent.begin(), ent.end());
            const int32_t lane = i - i0;
            for (int32_t k = 0; k < W; ++k) m->sell_col[((size_t)s * W + k) * kBlock + lane] = i;
            for (size_t e = 0; e < ent.size(); ++e) {
                int32_t k = (int32_t)e;
                if (regular)
                    k = (int32_t)(std::lower_bound(offs.begin(), offs.end(), ent[e].first - i) - offs.begin());
                const size_t at = ((size_t)s * W + k) * kBlock + lane;
                m->sell_fe[at] = ent[e].second;
                m->sell_col[at] = ent[e].first;
            }
        }
    }
    // mirror slots of the regular slices (the matrix is symmetric in
    // structure and value: entry (i, j) of slot k equals entry (j, i), which a
    // regular neighbour slice holds in the slot whose offset is -off_k)
    m->sell_mir.assign((size_t)ns * W, -1);
    // a slot is real if some cell of the slice has an entry there
    std::vector<char> used((size_t)ns * W, 0);
    for (int32_t s = 0; s < ns; ++s)
        for (int32_t k = 0; k < W; ++k)
            for (int32_t l = 0; l < kBlock && !used[(size_t)s * W + k]; ++l)
                used[(size_t)s * W + k] = m->sell_fe[((size_t)s * W + k) * kBlock + l] >= 0;
    auto slot_of = [&](int32_t s, int32_t off) {
        if (s < 0 || s >= ns || m->sell_mode[s] != 0) return -1;
        for (int32_t k = 0; k < W; ++k)
            if (used[(size_t)s * W + k] && m->sell_off[(size_t)s * W + k] == off) return k;
        return -1;
    };
    for (int32_t s = 0; s < ns; ++s) {
        if (m->sell_mode[s] != 0) continue;
        const int32_t i0 = s * kBlock, i1 = std::min(N, i0 + kBlock);
        for (int32_t k = 0; k < W; ++k) {
            const int32_t off = m->sell_off[(size_t)s * W + k];
            if (off >= 0 || !used[(size_t)s * W + k] || i0 + off < 0) continue;
            // the neighbours j = i + off of the slice's cells span at most two slices
            const int32_t sa = (i0 + off) / kBlock, sb = (i1 - 1 + off) / kBlock;
            const int32_t ka = slot_of(sa, -off);
            if (ka < 0 || (sb != sa && slot_of(sb, -off) != ka)) continue;
            // every entry of slot k must be the mirror of the neighbour's entry
            // (padding on both sides, or the same face)
            bool ok = true;
            for (int32_t i = i0; i < i1 && ok; ++i) {
                const int32_t j = i + off;
                const int32_t fe = m->sell_fe[((size_t)s * W + k) * kBlock + (i - i0)];
                const int32_t fm = m->sell_fe[((size_t)(j / kBlock) * W + ka) * kBlock + (j % kBlock)];
                ok = (fe < 0 && fm < 0) || (fe >= 0 && fm >= 0 && (fe >> 1) == (fm >> 1));
            }
            if (ok) m->sell_mir[(size_t)s * W + k] = ka;
        }
    }
    // slices of the 7-point form (the test the paired product makes per
    // slice on the device)
    m->sell_n7 = 0;
    if (W == 6)
        for (int32_t s = 0; s < ns; ++s) {
            if (m->sell_mode[s] != 0) continue;
            const int32_t *o = &m->sell_off[(size_t)s * 6], *mr = &m->sell_mir[(size_t)s * 6];
            const int32_t b = o[4], c = o[5];
            const int64_t lo = (int64_t)s * kBlock;
            const bool ok = o[2] == -1 && o[3] == 1 && o[1] == -b && o[0] == -c && b > 1 && c > b &&
                            ((b | c) & 1) == 0 && mr[0] == 5 && mr[1] == 4 && mr[2] == 3 && mr[3] < 0 && mr[4] < 0 &&
                            mr[5] < 0 && lo - c >= 0 && lo + kBlock - 1 + c <= (int64_t)N - 1;
            m->sell_n7 += ok ? 1 : 0;
        }
}

}  // namespace

// Hybrid layout (Section 3.1).  Row i in ascending column order is: the
// owners of the faces whose neighbour is i (losort order: ascending owner),
// the diagonal, the neighbours of the faces i owns (ascending neighbour).
// So the slot of every entry follows from face positions alone: face f =
// (o, n), o < n, sits at slot nlow(o) + 1 + (f - own_start[o]) of row o and
// at slot (t - nbr_start[n]) of row n, where losort[t] = f.
void build_hybrid(const fvm_mesh &m, int32_t K, HybridHost &h)
{
    const int32_t N = m.N, Fi = m.Fi;
    h.K = K;
    std::vector<int32_t> nlow(N), len(N);
    for (int32_t i = 0; i < N; ++i) {
        nlow[i] = m.nbr_start[i + 1] - m.nbr_start[i];
        len[i] = nlow[i] + 1 + (m.own_start[i + 1] - m.own_start[i]);
    }
    h.c_start.assign((size_t)N + 1, 0);
    for (int32_t i = 0; i < N; ++i) h.c_start[i + 1] = h.c_start[i] + std::max(0, len[i] - K);
    h.nC = h.c_start[N];
    std::vector<int32_t> lpos(Fi);
    for (int32_t t = 0; t < Fi; ++t) lpos[m.losort[t]] = t;
    // an entry (row, slot): its paper-form transpose code and device position
    auto code = [&](int32_t row, int32_t slot) { return slot < K ? slot : -1 - (h.c_start[row] + slot - K); };
    auto devpos = [&](int32_t row, int32_t slot) {
        return slot < K ? (int32_t)((int64_t)slot * N + row) : (int32_t)((int64_t)K * N + h.c_start[row] + slot - K);
    };
    h.I.assign((size_t)N * K, 0);
    h.J.assign((size_t)N * K, 0);
    for (int32_t i = 0; i < N; ++i)
        for (int32_t k = 0; k < K; ++k) {   // unused slots; real entries are overwritten below
            h.I[(size_t)i * K + k] = i;
            h.J[(size_t)i * K + k] = k;
        }
    h.c_col.assign(h.nC, 0);
    h.c_tr.assign(h.nC, 0);
    h.dpos.assign(N, 0);
    h.locO.assign(Fi, 0);
    h.locN.assign(Fi, 0);
    // place one entry: row r, slot sl, column col, transpose at (tr_row, tr_slot)
    auto place = [&](int32_t r, int32_t sl, int32_t col, int32_t tr_row, int32_t tr_slot) {
        if (sl < K) {
            h.I[(size_t)r * K + sl] = col;
            h.J[(size_t)r * K + sl] = code(tr_row, tr_slot);
        } else {
            const int32_t c = h.c_start[r] + sl - K;
            h.c_col[c] = col;
            h.c_tr[c] = tr_slot < K ? K * tr_row + tr_slot : code(tr_row, tr_slot);
        }
    };
    for (int32_t i = 0; i < N; ++i) {
        place(i, nlow[i], i, i, nlow[i]);
        h.dpos[i] = devpos(i, nlow[i]);
    }
    for (int32_t o = 0; o < N; ++o)
        for (int32_t f = m.own_start[o]; f < m.own_start[o + 1]; ++f) {
            const int32_t n = m.nei[f];
            const int32_t so = nlow[o] + 1 + (f - m.own_start[o]);
            const int32_t sn = lpos[f] - m.nbr_start[n];
            place(o, so, n, n, sn);
            place(n, sn, o, o, so);
            h.locO[f] = devpos(o, so);
            h.locN[f] = devpos(n, sn);
        }
    // device forms
    h.dI.assign((size_t)N * K, 0);
    h.dJ.assign((size_t)N * K, 0);
    for (int32_t i = 0; i < N; ++i)
        for (int32_t k = 0; k < K; ++k) {
            h.dI[(size_t)k * N + i] = h.I[(size_t)i * K + k];
            h.dJ[(size_t)k * N + i] = h.J[(size_t)i * K + k];
        }
    h.c_trpos.assign(h.nC, 0);
    for (int32_t c = 0; c < h.nC; ++c) {
        const int32_t t = h.c_tr[c];
        h.c_trpos[c] = t >= 0 ? (int32_t)((int64_t)(t % K) * N + t / K) : (int32_t)((int64_t)K * N + (-1 - t));
    }
}

// AMG hierarchy.  Aggregation of a level in cell index order: a cell none
// of whose neighbours is aggregated yet starts an aggregate with all of them;
// every cell left over joins the aggregate of its lowest-index neighbour
// aggregated that way (a cell without neighbours is its own aggregate).
// Levels are added while a level has more than kAmgCoarseMax cells and the
// aggregation shrinks it by at least 10%.
namespace {

// neighbour-side faces of cell i in losort order, then owned faces: the
// neighbours in ascending order
template <class Fn>
void for_neighbours(const std::vector<int32_t> &own, const std::vector<int32_t> &nei,
                    const std::vector<int32_t> &own_start, const std::vector<int32_t> &nbr_start,
                    const std::vector<int32_t> &losort, int32_t i, Fn fn)
{
    for (int32_t k = nbr_start[i]; k < nbr_start[i + 1]; ++k) fn(own[losort[k]]);
    for (int32_t f = own_start[i]; f < own_start[i + 1]; ++f) fn(nei[f]);
}

void face_ranges(int32_t n, const std::vector<int32_t> &own, const std::vector<int32_t> &nei,
                 std::vector<int32_t> &own_start, std::vector<int32_t> &nbr_start, std::vector<int32_t> &losort)
{
    const int32_t nf = (int32_t)nei.size();
    own_start.assign((size_t)n + 1, 0);
    nbr_start.assign((size_t)n + 1, 0);
    for (int32_t f = 0; f < nf; ++f) { own_start[own[f] + 1]++; nbr_start[nei[f] + 1]++; }
    for (int32_t i = 0; i < n; ++i) { own_start[i + 1] += own_start[i]; nbr_start[i + 1] += nbr_start[i]; }
    losort.assign(nf, 0);
    std::vector<int32_t> fill(nbr_start.begin(), nbr_start.end() - 1);
    for (int32_t f = 0; f < nf; ++f) losort[fill[nei[f]]++] = f;   // faces ascending: owners ascending per cell
}

}  // namespace

const AmgHost &mesh_amg(const fvm_mesh &m)
{
    if (m.amg) return *m.amg;
    auto h = std::make_shared<AmgHost>();
    h->L.emplace_back();
    {
        AmgLevelHost &L0 = h->L[0];
        L0.n = m.N;
        L0.nf = m.Fi;
    }
    // level 0 topology is the mesh's
    const std::vector<int32_t> own0(m.own.begin(), m.own.begin() + m.Fi);
    const std::vector<int32_t> *own = &own0, *nei = &m.nei, *os = &m.own_start, *ns = &m.nbr_start, *lo = &m.losort;
    while (h->L.back().n > kAmgCoarseMax && h->L.size() < 20) {
        const int32_t l = (int32_t)h->L.size() - 1;
        const int32_t n = h->L[l].n;
        std::vector<int32_t> agg(n, -1);
        std::vector<char> first(n, 0);
        int32_t na = 0;
        for (int32_t i = 0; i < n; ++i) {
            if (agg[i] != -1) continue;
            bool free_all = true;
            for_neighbours(*own, *nei, *os, *ns, *lo, i, [&](int32_t j) { free_all = free_all && agg[j] == -1; });
            if (!free_all) continue;
            agg[i] = na;
            first[i] = 1;
            for_neighbours(*own, *nei, *os, *ns, *lo, i, [&](int32_t j) { agg[j] = na; first[j] = 1; });
            ++na;
        }
        for (int32_t i = 0; i < n; ++i) {
            if (agg[i] != -1) continue;
            int32_t to = -1;
            for_neighbours(*own, *nei, *os, *ns, *lo, i, [&](int32_t j) { if (to < 0 && first[j]) to = agg[j]; });
            agg[i] = to >= 0 ? to : na++;
        }
        if (na > 0.9 * n) break;
        // coarse faces: distinct aggregate pairs, sorted
        const int32_t nf = (int32_t)nei->size();
        std::vector<int64_t> key;
        key.reserve(nf);
        for (int32_t f = 0; f < nf; ++f) {
            const int32_t A = agg[(*own)[f]], B = agg[(*nei)[f]];
            if (A != B) key.push_back((int64_t)std::min(A, B) * na + std::max(A, B));
        }
        std::sort(key.begin(), key.end());
        key.erase(std::unique(key.begin(), key.end()), key.end());
        AmgLevelHost C;
        C.n = na;
        C.nf = (int32_t)key.size();
        C.own.resize(C.nf);
        C.nei.resize(C.nf);
        for (int32_t F = 0; F < C.nf; ++F) { C.own[F] = (int32_t)(key[F] / na); C.nei[F] = (int32_t)(key[F] % na); }
        face_ranges(C.n, C.own, C.nei, C.own_start, C.nbr_start, C.losort);
        // gather lists (ascending fine index)
        C.mstart.assign((size_t)na + 1, 0);
        for (int32_t i = 0; i < n; ++i) C.mstart[agg[i] + 1]++;
        for (int32_t a = 0; a < na; ++a) C.mstart[a + 1] += C.mstart[a];
        C.members.resize(n);
        {
            std::vector<int32_t> fill(C.mstart.begin(), C.mstart.end() - 1);
            for (int32_t i = 0; i < n; ++i) C.members[fill[agg[i]]++] = i;
        }
        C.istart.assign((size_t)na + 1, 0);
        C.cstart.assign((size_t)C.nf + 1, 0);
        std::vector<int32_t> cf(nf, -1);
        for (int32_t f = 0; f < nf; ++f) {
            const int32_t A = agg[(*own)[f]], B = agg[(*nei)[f]];
            if (A == B) C.istart[A + 1]++;
            else {
                const int64_t k = (int64_t)std::min(A, B) * na + std::max(A, B);
                cf[f] = (int32_t)(std::lower_bound(key.begin(), key.end(), k) - key.begin());
                C.cstart[cf[f] + 1]++;
            }
        }
        for (int32_t a = 0; a < na; ++a) C.istart[a + 1] += C.istart[a];
        for (int32_t F = 0; F < C.nf; ++F) C.cstart[F + 1] += C.cstart[F];
        C.inner.resize(C.istart[na]);
        C.cfaces.resize(C.cstart[C.nf]);
        {
            std::vector<int32_t> fi(C.istart.begin(), C.istart.end() - 1), fc(C.cstart.begin(), C.cstart.end() - 1);
            for (int32_t f = 0; f < nf; ++f) {
                if (cf[f] < 0) C.inner[fi[agg[(*own)[f]]]++] = f;
                else C.cfaces[fc[cf[f]]++] = f;
            }
        }
        h->L[l].agg = std::move(agg);
        h->L.push_back(std::move(C));
        const AmgLevelHost &N = h->L.back();
        own = &N.own; nei = &N.nei; os = &N.own_start; ns = &N.nbr_start; lo = &N.losort;
    }
    m.amg = h;
    return *h;
}

namespace {

fvm_status build(const fvm_mesh_desc *d, fvm_mesh *m)
{
    if (!d || d->n_cells < 1 || d->n_internal_faces < 0 || d->n_faces < d->n_internal_faces || d->n_patches < 0)
        return fvm_fail(FVM_EINVAL, "mesh: bad sizes");
    if (!d->owner || (d->n_internal_faces > 0 && !d->neighbour) || !d->Sf || !d->Cf || !d->C || !d->V ||
        (d->n_patches > 0 && !d->patches))
        return fvm_fail(FVM_EINVAL, "mesh: null array");
    const int32_t N = d->n_cells, F = d->n_faces, Fi = d->n_internal_faces, Fb = F - Fi;
    m->N = N; m->F = F; m->Fi = Fi; m->Fb = Fb; m->npatch = d->n_patches;

    for (int32_t i = 0; i < N; ++i)
        if (!(d->V[i] > 0.0) || !std::isfinite(d->V[i]) || !finite3(d->C + 3 * (size_t)i))
            return fvm_fail(FVM_EINVAL, "mesh: cell " + std::to_string(i) + " has V <= 0 or non-finite geometry");
    for (int32_t f = 0; f < F; ++f) {
        if (d->owner[f] < 0 || d->owner[f] >= N)
            return fvm_fail(FVM_EINVAL, "mesh: owner out of range at face " + std::to_string(f));
        if (!finite3(d->Sf + 3 * (size_t)f) || !finite3(d->Cf + 3 * (size_t)f))
            return fvm_fail(FVM_EINVAL, "mesh: non-finite face geometry at face " + std::to_string(f));
    }
    for (int32_t f = 0; f < Fi; ++f) {
        if (d->neighbour[f] < 0 || d->neighbour[f] >= N)
            return fvm_fail(FVM_EINVAL, "mesh: neighbour out of range at face " + std::to_string(f));
        if (d->neighbour[f] == d->owner[f])
            return fvm_fail(FVM_EINVAL, "mesh: owner == neighbour at face " + std::to_string(f));
    }
    // patches must tile the boundary faces in order
    int32_t expect = Fi;
    m->patches.assign(d->patches, d->patches + d->n_patches);
    for (int32_t p = 0; p < d->n_patches; ++p) {
        const fvm_patch &P = d->patches[p];
        if (P.start != expect || P.size < 0)
            return fvm_fail(FVM_EINVAL, "mesh: patches do not tile the boundary faces (patch " + std::to_string(p) + ")");
        if (P.u_kind < 0 || P.u_kind > 2 || P.p_kind < 0 || P.p_kind > 2)
            return fvm_fail(FVM_EINVAL, "mesh: unknown boundary kind in patch " + std::to_string(p));
        expect += P.size;
        if (P.p_kind == FVM_BC_FIXED && P.size > 0) m->has_fixed_p = true;
    }
    if (expect != F) return fvm_fail(FVM_EINVAL, "mesh: boundary faces without a patch");

    // orientation test S.d > 0 in the caller's orientation
    auto sd_int = [&](int32_t f) {
        const double *S = d->Sf + 3 * (size_t)f, *CP = d->C + 3 * (size_t)d->owner[f], *CN = d->C + 3 * (size_t)d->neighbour[f];
        return S[0] * (CN[0] - CP[0]) + S[1] * (CN[1] - CP[1]) + S[2] * (CN[2] - CP[2]);
    };
    for (int32_t f = 0; f < Fi; ++f)
        if (!(sd_int(f) > 0.0)) return fvm_fail(FVM_EINVAL, "mesh: S.d <= 0 at internal face " + std::to_string(f));
    for (int32_t f = Fi; f < F; ++f) {
        const double *S = d->Sf + 3 * (size_t)f, *Cf = d->Cf + 3 * (size_t)f, *CP = d->C + 3 * (size_t)d->owner[f];
        double sd = S[0] * (Cf[0] - CP[0]) + S[1] * (Cf[1] - CP[1]) + S[2] * (Cf[2] - CP[2]);
        if (!(sd > 0.0)) return fvm_fail(FVM_EINVAL, "mesh: S.d <= 0 at boundary face " + std::to_string(f));
    }

    // canonical internal faces: bucket by lower cell, then by upper cell
    std::vector<int32_t> lo(Fi), hi(Fi);
    m->own_start.assign((size_t)N + 1, 0);
    for (int32_t f = 0; f < Fi; ++f) {
        int32_t a = d->owner[f], b = d->neighbour[f];
        lo[f] = std::min(a, b); hi[f] = std::max(a, b);
        m->own_start[lo[f] + 1]++;
    }
    for (int32_t i = 0; i < N; ++i) m->own_start[i + 1] += m->own_start[i];
    std::vector<int32_t> order(Fi), fill(m->own_start.begin(), m->own_start.end() - 1);
    for (int32_t f = 0; f < Fi; ++f) order[fill[lo[f]]++] = f;
    for (int32_t i = 0; i < N; ++i) {
        auto b = order.begin() + m->own_start[i], e = order.begin() + m->own_start[i + 1];
        std::sort(b, e, [&](int32_t x, int32_t y) { return hi[x] < hi[y] || (hi[x] == hi[y] && x < y); });
        for (auto it = b; it + 1 < e; ++it)
            if (hi[*it] == hi[*(it + 1)])
                return fvm_fail(FVM_EINVAL, "mesh: duplicated face between cells " + std::to_string(i) + " and " +
                                                std::to_string(hi[*it]));
    }
    m->own.resize(F); m->nei.resize(Fi); m->face_user.resize(Fi); m->face_sign.resize(Fi);
    for (int32_t f = Fi; f < F; ++f) m->own[f] = d->owner[f];   // boundary faces keep the caller's order
    for (int32_t c = 0; c < Fi; ++c) {
        int32_t f = order[c];
        m->own[c] = lo[f]; m->nei[c] = hi[f]; m->face_user[c] = f;
        m->face_sign[c] = d->owner[f] == lo[f] ? 1 : -1;
    }
    // neighbour-side index: faces ordered by (nei, own); filling buckets in
    // canonical order keeps each bucket sorted by owner
    m->nbr_start.assign((size_t)N + 1, 0);
    for (int32_t c = 0; c < Fi; ++c) m->nbr_start[m->nei[c] + 1]++;
    for (int32_t i = 0; i < N; ++i) m->nbr_start[i + 1] += m->nbr_start[i];
    m->losort.resize(Fi);
    fill.assign(m->nbr_start.begin(), m->nbr_start.end() - 1);
    for (int32_t c = 0; c < Fi; ++c) m->losort[fill[m->nei[c]]++] = c;
    // boundary faces by cell
    m->bnd_start.assign((size_t)N + 1, 0);
    m->bpatch.resize(Fb);
    for (int32_t p = 0; p < d->n_patches; ++p)
        for (int32_t k = 0; k < d->patches[p].size; ++k) m->bpatch[d->patches[p].start + k - Fi] = p;
    for (int32_t b = 0; b < Fb; ++b) m->bnd_start[d->owner[Fi + b] + 1]++;
    for (int32_t i = 0; i < N; ++i) m->bnd_start[i + 1] += m->bnd_start[i];
    m->bnd_list.resize(Fb);
    fill.assign(m->bnd_start.begin(), m->bnd_start.end() - 1);
    for (int32_t b = 0; b < Fb; ++b) m->bnd_list[fill[d->owner[Fi + b]]++] = b;

    // geometry, SoA, canonical orientation
    m->S.resize(3 * (size_t)F); m->Cf.resize(3 * (size_t)F); m->C.resize(3 * (size_t)N); m->V.assign(d->V, d->V + N);
    for (int32_t c = 0; c < F; ++c) {
        int32_t f = c < Fi ? m->face_user[c] : c;
        double sg = c < Fi ? (double)m->face_sign[c] : 1.0;
        for (int k = 0; k < 3; ++k) {
            m->S[(size_t)k * F + c] = sg * d->Sf[3 * (size_t)f + k];
            m->Cf[(size_t)k * F + c] = d->Cf[3 * (size_t)f + k];
        }
    }
    for (int32_t i = 0; i < N; ++i)
        for (int k = 0; k < 3; ++k) m->C[(size_t)k * N + i] = d->C[3 * (size_t)i + k];

    // orthogonality: sine of the angle between S and d above 1e-8 anywhere
    m->nonorth = false;
    for (int32_t c = 0; c < Fi && !m->nonorth; ++c) {
        double S[3], dd[3];
        for (int k = 0; k < 3; ++k) {
            S[k] = m->S[(size_t)k * F + c];
            dd[k] = m->C[(size_t)k * N + m->nei[c]] - m->C[(size_t)k * N + m->own[c]];
        }
        double cx = S[1] * dd[2] - S[2] * dd[1], cy = S[2] * dd[0] - S[0] * dd[2], cz = S[0] * dd[1] - S[1] * dd[0];
        double s2 = cx * cx + cy * cy + cz * cz;
        double n2 = (S[0] * S[0] + S[1] * S[1] + S[2] * S[2]) * (dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
        if (s2 > 1e-16 * n2) m->nonorth = true;
    }

    // level schedule of the lower-triangular dependency graph: level(i) =
    // 1 + max level of its lower neighbours j < i (ascending i)
    std::vector<int32_t> lev(N, 0);
    int32_t nl = 0;
    for (int32_t i = 0; i < N; ++i) {
        int32_t l = 0;
        for (int32_t k = m->nbr_start[i]; k < m->nbr_start[i + 1]; ++k) l = std::max(l, lev[m->own[m->losort[k]]] + 1);
        lev[i] = l;
        nl = std::max(nl, l + 1);
    }
    m->lvl_start.assign((size_t)nl + 1, 0);
    for (int32_t i = 0; i < N; ++i) m->lvl_start[lev[i] + 1]++;
    for (int32_t l = 0; l < nl; ++l) m->lvl_start[l + 1] += m->lvl_start[l];
    m->lvl_cells.resize(N);
    fill.assign(m->lvl_start.begin(), m->lvl_start.end() - 1);
    for (int32_t i = 0; i < N; ++i) m->lvl_cells[fill[lev[i]]++] = i;
    m->lvl_pos.resize(N);
    for (int32_t k = 0; k < N; ++k) m->lvl_pos[m->lvl_cells[k]] = k;
    m->lvl_of = lev;
    // dependencies in level order
    {
        int32_t wl = 0, wh = 0;
        for (int32_t i = 0; i < N; ++i) {
            wl = std::max(wl, m->nbr_start[i + 1] - m->nbr_start[i]);
            wh = std::max(wh, m->own_start[i + 1] - m->own_start[i]);
        }
        m->dW_lo = std::max(wl, 1);
        m->dW_hi = std::max(wh, 1);
        m->dl_pos.assign((size_t)m->dW_lo * N, -1); m->dl_face.assign((size_t)m->dW_lo * N, -1);
        m->du_pos.assign((size_t)m->dW_hi * N, -1); m->du_face.assign((size_t)m->dW_hi * N, -1);
        for (int32_t q = 0; q < N; ++q) {
            const int32_t i = m->lvl_cells[q];
            int32_t k = 0;
            for (int32_t t = m->nbr_start[i]; t < m->nbr_start[i + 1]; ++t, ++k) {
                const int32_t f = m->losort[t];
                m->dl_pos[(size_t)k * N + q] = m->lvl_pos[m->own[f]];
                m->dl_face[(size_t)k * N + q] = f;
            }
            k = 0;
            for (int32_t f = m->own_start[i]; f < m->own_start[i + 1]; ++f, ++k) {
                m->du_pos[(size_t)k * N + q] = m->lvl_pos[m->nei[f]];
                m->du_face[(size_t)k * N + q] = f;
            }
        }
    }
    build_sell(m);
    return FVM_OK;
}

}  // namespace

extern "C" fvm_status fvm_mesh_create(const fvm_mesh_desc *desc, fvm_mesh **out)
{
    if (!out) return fvm_fail(FVM_EINVAL, "mesh: null output");
    *out = nullptr;
    fvm_mesh *m = new (std::nothrow) fvm_mesh();
    if (!m) return fvm_fail(FVM_EINVAL, "mesh: out of host memory");
    fvm_status st;
    try {
        st = build(desc, m);
    } catch (const std::exception &e) {
        st = fvm_fail(FVM_EINVAL, std::string("mesh: ") + e.what());
    }
    if (st != FVM_OK) {
        delete m;
        return st;
    }
    *out = m;
    return FVM_OK;
}

extern "C" void fvm_mesh_destroy(fvm_mesh *mesh) { delete mesh; }

extern "C" fvm_status fvm_mesh_amg(const fvm_mesh *m, int32_t level, int32_t *n_levels, int32_t *n_cells,
                                   int32_t *n_faces, int32_t *own, int32_t *nei, int32_t *agg)
{
    if (!m) return fvm_fail(FVM_EINVAL, "amg: null mesh");
    try {
        const AmgHost &h = mesh_amg(*m);
        const int32_t nl = (int32_t)h.L.size();
        if (n_levels) *n_levels = nl;
        if (level < 0 || level >= nl) return fvm_fail(FVM_EINVAL, "amg: level out of range");
        const AmgLevelHost &L = h.L[level];
        if (n_cells) *n_cells = L.n;
        if (n_faces) *n_faces = L.nf;
        if (level == 0) {
            if (own) std::copy(m->own.begin(), m->own.begin() + m->Fi, own);
            if (nei) std::copy(m->nei.begin(), m->nei.end(), nei);
        } else {
            if (own) std::copy(L.own.begin(), L.own.end(), own);
            if (nei) std::copy(L.nei.begin(), L.nei.end(), nei);
        }
        if (agg && level < nl - 1) std::copy(L.agg.begin(), L.agg.end(), agg);
    } catch (const std::bad_alloc &) {
        return fvm_fail(FVM_ENOMEM, "amg: out of host memory");
    }
    return FVM_OK;
}

extern "C" fvm_status fvm_mesh_hybrid(const fvm_mesh *m, int32_t K, int32_t *n_crs, int32_t *I, int32_t *J,
                                      int32_t *Q, int32_t *c_start, int32_t *c_col, int32_t *c_tr)
{
    if (!m) return fvm_fail(FVM_EINVAL, "hybrid: null mesh");
    if (K < 1) return fvm_fail(FVM_EINVAL, "hybrid: K must be >= 1");
    if ((int64_t)K * m->N >= INT32_MAX) return fvm_fail(FVM_EINVAL, "hybrid: K * n_cells exceeds int32");
    try {
        HybridHost h;
        build_hybrid(*m, K, h);
        if (n_crs) *n_crs = h.nC;
        const size_t NK = (size_t)m->N * K;
        if (I) std::copy(h.I.begin(), h.I.end(), I);
        if (J) std::copy(h.J.begin(), h.J.end(), J);
        if (Q)
            for (size_t e = 0; e < NK; ++e) Q[e] = h.J[e] >= 0 ? K * h.I[e] + h.J[e] : -1;
        if (c_start) std::copy(h.c_start.begin(), h.c_start.end(), c_start);
        if (c_col) std::copy(h.c_col.begin(), h.c_col.end(), c_col);
        if (c_tr) std::copy(h.c_tr.begin(), h.c_tr.end(), c_tr);
    } catch (const std::bad_alloc &) {
        return fvm_fail(FVM_ENOMEM, "hybrid: out of host memory");
    }
    return FVM_OK;
}

extern "C" fvm_status fvm_mesh_info(const fvm_mesh *m, int32_t *n_cells, int32_t *n_faces, int32_t *n_internal,
                                    int32_t *non_orthogonal)
{
    if (!m) return fvm_fail(FVM_EINVAL, "mesh: null handle");
    if (n_cells) *n_cells = m->N;
    if (n_faces) *n_faces = m->F;
    if (n_internal) *n_internal = m->Fi;
    if (non_orthogonal) *non_orthogonal = m->nonorth ? 1 : 0;
    return FVM_OK;
}

extern "C" fvm_status fvm_mesh_sell_info(const fvm_mesh *m, int32_t *w_slots, int32_t *n_slices,
                                         int32_t *n_explicit_slices, int64_t *explicit_entries,
                                         int64_t *mirrored_entries, int32_t *n_7pt_slices)
{
    if (!m) return fvm_fail(FVM_EINVAL, "mesh: null handle");
    const int32_t W = m->sell_W, ns = (int32_t)m->sell_mode.size();
    int32_t nx = 0;
    int64_t ex = 0, mir = 0;
    for (int32_t s = 0; s < ns; ++s) {
        const bool explicit_cols = m->sell_mode[s] != 0;
        nx += explicit_cols ? 1 : 0;
        for (int32_t k = 0; k < W; ++k) {
            int64_t used = 0;
            for (int32_t l = 0; l < kBlock; ++l) used += m->sell_fe[((size_t)s * W + k) * kBlock + l] >= 0;
            if (explicit_cols) ex += used;
            else if (m->sell_mir[(size_t)s * W + k] >= 0) mir += used;
        }
    }
    if (w_slots) *w_slots = W;
    if (n_slices) *n_slices = ns;
    if (n_explicit_slices) *n_explicit_slices = nx;
    if (explicit_entries) *explicit_entries = ex;
    if (mirrored_entries) *mirrored_entries = mir;
    if (n_7pt_slices) *n_7pt_slices = m->sell_n7;
    return FVM_OK;
}
