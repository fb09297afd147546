"""Host-side mesh preparation (no GPU): the sliced-ELL face lists and the
tile tables of the fused transport kernel, read back from a host-only mesh
and checked against the mesh they were built from."""
import numpy as np
import pytest

import rtgen
from paper_2404_17630_amd import rt

SLICE, TILE = 64, rt.RT_TILE_CELLS
TILE_SLICES = TILE // SLICE


def meshes():
    return {
        "lattice_ragged_hilbert": rtgen.jittered_lattice((12, 10, 9), 1.0, 0.2, 3, "hilbert").as_dict(),
        "lattice_random": rtgen.jittered_lattice((9, 8, 7), 1.0, 0.2, 3, "random").as_dict(),
        "bcc_hilbert": rtgen.staggered_bcc(5, 1.0, 0.1, 4, "hilbert").as_dict(),
        "lattice_small": rtgen.jittered_lattice((3, 3, 3), 1.0, 0.1, 2, "lattice").as_dict(),
        "split_faces": rtgen.split_faces(rtgen.jittered_lattice((10, 9, 8), 1.0, 0.2, 3, "hilbert"), 0.2, 5).as_dict(),
    }


@pytest.fixture(scope="module", params=list(meshes()))
def mesh(request):
    m = meshes()[request.param]
    h = rt.Mesh(m, device=rt.RT_DEVICE_HOST_ONLY)
    tabs = {name: h.table(name) for name in rt.TABLES}
    h.close()
    return m, tabs


def entries_of(tabs, nc):
    """cell -> list of (entry, slot) from the sliced ELL."""
    sptr, sdeg = tabs["sptr"], tabs["sdeg"]
    out = []
    for i in range(nc):
        s = i // SLICE
        out.append([(sptr[s] + k * SLICE + i % SLICE, k) for k in range(sdeg[s])])
    return out


def test_sliced_ell_matches_faces(mesh):
    m, t = mesh
    nc, nf = m["n_cells"], m["n_faces"]
    fc = m["face_cells"]
    ent = entries_of(t, nc)
    seen = np.zeros((2, nf), int)
    for i in range(nc):
        faces = []
        for e, _ in ent[i]:
            j = t["nbr"][e]
            if j < 0:
                continue
            fs = t["fsf"][e]
            f = fs if fs >= 0 else ~fs
            side = 0 if fs >= 0 else 1
            assert fc[side, f] == i and fc[1 - side, f] == j
            seen[side, f] += 1
            faces.append(f)
            # the opposite entry is the same face seen from the neighbour
            eo = t["opp"][e]
            assert t["nbr"][eo] == i and t["opp"][eo] == e
            assert (t["fsf"][eo] if t["fsf"][eo] >= 0 else ~t["fsf"][eo]) == f
        assert faces == sorted(faces)          # face-index order within a cell
    assert np.all(seen == 1)


def test_tile_tables_route_every_opposite_state(mesh):
    """Every face side of a tile cell finds the state on the other side of its
    face in an LDS slot that exactly one work item writes: the neighbour's own
    entry when it is in the tile, else the halo side listed for it."""
    m, t = mesh
    nc = m["n_cells"]
    sptr, nbr, opp = t["sptr"], t["nbr"], t["opp"]
    ns = len(t["sdeg"])
    ntiles = (nc + TILE - 1) // TILE
    assert len(t["halo_ptr"]) == ntiles + 1 and t["halo_ptr"][0] == 0
    assert len(t["hside_ptr"]) == len(t["halo_cell"]) + 1
    cell_of_entry = np.full(len(nbr), -1)
    for i, lst in enumerate(entries_of(t, nc)):
        for e, _ in lst:
            cell_of_entry[e] = i
    for tt in range(ntiles):
        c0, c1 = tt * TILE, min(nc, tt * TILE + TILE)
        e0 = sptr[tt * TILE_SLICES]
        n_own = sptr[min(ns, (tt + 1) * TILE_SLICES)] - e0
        q0, q1 = t["halo_ptr"][tt], t["halo_ptr"][tt + 1]
        hs0, hs1 = t["hside_ptr"][q0], t["hside_ptr"][q1]
        writes = np.zeros(n_own + (hs1 - hs0), int)
        # own slots: every real entry of a tile cell
        for e in range(e0, e0 + n_own):
            if nbr[e] >= 0 and c0 <= cell_of_entry[e] < c1:
                writes[e - e0] += 1
        # halo slots
        halo = t["halo_cell"][q0:q1]
        assert np.all((halo < c0) | (halo >= c1))
        assert len(set(halo.tolist())) == len(halo)
        for q in range(q0, q1):
            for s in range(t["hside_ptr"][q], t["hside_ptr"][q + 1]):
                e = t["hside_entry"][s]
                assert cell_of_entry[e] == t["halo_cell"][q]
                assert c0 <= nbr[e] < c1            # the side faces a tile cell
                writes[n_own + s - hs0] += 1
        assert np.all(writes <= 1)
        # every tile entry reads a written slot holding its opposite state
        for i in range(c0, c1):
            for e, _ in entries_of(t, nc)[i]:
                if nbr[e] < 0:
                    continue
                slot = t["lds_opp"][e]
                assert 0 <= slot < len(writes) and writes[slot] == 1
                eo = opp[e]
                if c0 <= nbr[e] < c1:
                    assert slot == eo - e0
                else:
                    assert t["hside_entry"][hs0 + slot - n_own] == eo


def test_flux_items_evaluate_every_face_side_once(mesh):
    """The flux kernel's per-slice face evaluations on uniform-degree meshes:
    every face side of a slice's cells gets its product exactly once, either
    from its own evaluation or, for a face whose two sides are in the slice,
    negated from the L side's; an item's second value is the signed opposite
    entry.  A Hilbert-ordered lattice evaluates 240 of a 4x4x4 slice's 384
    sides."""
    m, tabs = mesh
    nc = m["n_cells"]
    sdeg, nbr, fsf, opp = tabs["sdeg"], tabs["nbr"], tabs["fsf"], tabs["opp"]
    ptr, items = tabs["fitem_ptr"], tabs["fitem"].reshape(-1, 2)
    uniform = sdeg.size > 0 and int(sdeg[0]) in (6, 14) and np.all(sdeg == sdeg[0])
    deg_ok = uniform and np.all(np.bincount(m["face_cells"].ravel(), minlength=nc) == sdeg[0])
    if not deg_ok:
        assert ptr.size == 0 and items.size == 0
        return
    per = int(sdeg[0]) * SLICE
    assert ptr.size == sdeg.size + 1 and ptr[0] == 0 and ptr[-1] == items.shape[0]
    pair_bit = 1 << 30
    for s in range(sdeg.size):
        got = np.zeros(per, int)
        for e_raw, os_ in items[ptr[s]:ptr[s + 1]]:
            pair = bool(e_raw & pair_bit)
            e = int(e_raw & ~pair_bit)
            assert e // per == s and nbr[e] >= 0
            assert os_ == (opp[e] if fsf[e] >= 0 else ~opp[e])
            got[e - s * per] += 1
            if pair:
                assert fsf[e] >= 0 and opp[e] // per == s
                got[opp[e] - s * per] += 1
            else:
                assert opp[e] // per != s
        valid = nbr[s * per:(s + 1) * per] >= 0
        assert np.array_equal(got, valid.astype(int)), s


def test_tile_faces_cover_every_face_side_once(mesh):
    """The split transport's faces by 256-cell tile on six-slot meshes: a
    face whose two sides are in one tile is listed once, as the (L, R) entry
    pair relative to the tile's first entry; every other face side is a
    boundary item, numbered in entry order, listed as (entry, opposite
    side's item, complemented for an R side), with the first item of every
    tile and slice.  Together they give every face side of the mesh its
    product exactly once, and the items of a cell follow from the slot masks
    of its slice as the kernels rank them (slot-major, then lane)."""
    m, tabs = mesh
    nc = m["n_cells"]
    sdeg, nbr, fsf, opp = tabs["sdeg"], tabs["nbr"], tabs["fsf"], tabs["opp"]
    pptr, pair, bptr, bnd = tabs["tpair_ptr"], tabs["tpair"], tabs["tbnd_ptr"], tabs["tbnd"].reshape(-1, 2)
    sptr_b = tabs["tbnd_sptr"]
    six = sdeg.size > 0 and np.all(sdeg == 6) and np.all(np.bincount(m["face_cells"].ravel(), minlength=nc) == 6)
    per, sper = 6 * TILE, 6 * SLICE
    if six:
        # the tile split is kept for compact tiles only: at most two
        # cross-tile sides per cell
        e_all = np.nonzero(nbr >= 0)[0]
        six = np.count_nonzero(opp[e_all] // per != e_all // per) <= 2 * nc
    if not six:
        assert pptr.size == 0 and pair.size == 0 and bptr.size == 0 and bnd.size == 0 and sptr_b.size == 0
        return
    nt, ns = (nc + TILE - 1) // TILE, sdeg.size
    assert pptr.size == nt + 1 and bptr.size == nt + 1 and sptr_b.size == ns + 1
    assert pptr[0] == 0 and pptr[-1] == pair.size and bptr[0] == 0 and bptr[-1] == bnd.shape[0]
    assert np.array_equal(bptr, sptr_b[np.minimum(np.arange(nt + 1) * TILE_SLICES, ns)])
    assert np.all(np.diff(bnd[:, 0]) > 0)                      # entry order
    got = np.zeros(nbr.size, int)
    for t in range(nt):
        e0 = t * per
        for p in pair[pptr[t]:pptr[t + 1]]:
            ql, qr = int(p) & 0xffff, int(p) >> 16
            assert fsf[e0 + ql] >= 0 and fsf[e0 + qr] < 0 and opp[e0 + ql] == e0 + qr
            got[e0 + ql] += 1
            got[e0 + qr] += 1
        for q in range(bptr[t], bptr[t + 1]):
            e, os_ = bnd[q]
            assert e // per == t and opp[e] // per != t
            o = os_ if fsf[e] >= 0 else ~os_
            assert bnd[o, 0] == opp[e] and bnd[o, 1] == (~q if fsf[e] >= 0 else q)
            got[e] += 1
    assert np.array_equal(got, (nbr >= 0).astype(int))
    # the kernels' ranking: per slice, slot-major then lane, from the masks
    item_of = {int(e): q for q, e in enumerate(bnd[:, 0])}
    for s in range(ns):
        r = sptr_b[s]
        for k in range(6):
            for lane in range(SLICE):
                e = s * sper + k * SLICE + lane
                if e in item_of:
                    assert item_of[e] == r
                    r += 1
        assert r == sptr_b[s + 1]


def test_hilbert_slice_of_a_lattice_evaluates_240_sides():
    m = rtgen.jittered_lattice((8, 8, 8), 1.0, 0.2, 3, "hilbert").as_dict()
    h = rt.Mesh(m, device=rt.RT_DEVICE_HOST_ONLY)
    ptr = h.table("fitem_ptr")
    h.close()
    assert np.all(np.diff(ptr) == 240)


def test_host_only_mesh_cannot_hold_a_state():
    cfg = rtgen.stromgren(n=4, n_sub=1)
    m = rt.Mesh(cfg["mesh"], device=rt.RT_DEVICE_HOST_ONLY)
    with pytest.raises(rt.RtError) as ei:
        rt.State.from_config(m, cfg)
    assert ei.value.code == rt.RT_EDEVICE
    m.close()


def _hub_mesh(n_spokes):
    """Cell 0 joined to cells 1..n; each of those also joined to its two
    neighbours on either side of a ring, so it has five faces."""
    n = n_spokes
    nc = n + 1
    L = [0] * n + list(range(1, n + 1)) * 2
    R = list(range(1, n + 1)) + [k % n + 1 for k in range(1, n + 1)] + [(k + 1) % n + 1 for k in range(1, n + 1)]
    nf = len(L)
    rng = np.random.default_rng(7)
    nrm = rng.normal(size=(3, nf))
    nrm /= np.linalg.norm(nrm, axis=0)
    return dict(n_cells=nc, volume=np.ones(nc), centre=rng.uniform(size=(3, nc)), n_faces=nf,
                face_cells=np.array([L, R], dtype=np.int64), area=np.ones(nf), normal=nrm,
                face_centre=rng.uniform(size=(3, nf)), box=np.zeros(3))


def test_mesh_rejects_a_cell_with_more_faces_than_the_kernels_count():
    """The per-block counters pack per-face counts in 21-bit fields, which
    holds for cells of up to 4096 faces; rt_mesh_create refuses more."""
    with pytest.raises(rt.RtError) as e:
        rt.Mesh(_hub_mesh(4097), device=rt.RT_DEVICE_HOST_ONLY)
    assert e.value.code == rt.RT_EMESH and "4097 faces (> 4096)" in str(e.value)


def test_mesh_rejects_a_cell_with_fewer_than_four_faces():
    m = _hub_mesh(8)
    # drop the second ring of faces: every ring cell is left with three
    keep = 2 * 8
    m["area"] = m["area"][:keep]
    m["face_cells"] = m["face_cells"][:, :keep]
    m["normal"] = m["normal"][:, :keep]
    m["face_centre"] = m["face_centre"][:, :keep]
    m["n_faces"] = keep
    with pytest.raises(rt.RtError) as e:
        rt.Mesh(m, device=rt.RT_DEVICE_HOST_ONLY)
    assert e.value.code == rt.RT_EMESH and "(< 4)" in str(e.value)
