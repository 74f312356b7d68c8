"""CPU emulation of the addressing of the tiled grid sweeps and of the
stage-two kernel that feeds them (no GPU).

For every grid shape the GPU tests and the benchmark use, the index
arithmetic of k_stage2_grid and k_ilu_grid (forward and backward, every
tile, lane and step, staging waves and the sweeping wave) is replayed in
numpy and checked against the sizes the library allocates:
- every load and store of the tile layouts, the face buffers, the solution
  z and the staging ring stays inside its buffer;
- the tile layouts are bijections of the grid's cells (each cell one slot,
  each slot at most one cell), forward and backward;
- the cell a sweep handles at (tile, step, lane) is the cell whose
  right-hand side the stage-two kernel wrote there, and the forward sweep's
  output lands in the backward step that handles the same cell;
- a face value polled by a tile is the one its neighbour tile published for
  the neighbouring cell (j - 1 or k - 1 forward, j + 1 or k + 1 backward), at
  a step that exists;
- without a first-stage result (cptr_ilu_solve alone) nothing reads e0.
The formulas mirror kernels.hip (grid_tile_slot, GridTile, k_ilu_grid's
staging loop, k_stage2_grid).  A GPU fault of an earlier version -- the
backward sweep reading e0 through a null pointer when M2^-1 ran alone -- is
the last item.
"""
import numpy as np
import pytest

TJ, TK = 16, 4
FACE = 3 * (TK + TJ)
SKJ, SKK = TJ - 1, TK - 1

SHAPES = [(20, 20, 5), (7, 5, 3), (33, 17, 2), (2, 2, 2), (9, 7, 3), (3, 3, 2), (100, 100, 20),
          (30, 20, 6), (12, 10, 4), (16, 16, 8), (6, 5, 4), (40, 40, 10), (80, 80, 20), (160, 160, 20),
          (200, 200, 40), (250, 250, 50), (250, 250, 2), (60, 60, 8)]
# staging waves and ring slots (kernels.hip defaults)
CONFIGS = {True: (5, 6), False: (3, 4)}


def layout(nx, ny, nz):
    nJ, nK = -(-ny // TJ), -(-nz // TK)
    ns = nx + SKJ + SKK
    return nJ, nK, ns, nJ * nK, nJ * nK * ns


def stage2_slots(nx, ny, nz):
    """k_stage2_grid: forward and backward rows and lanes of every cell."""
    nJ, nK, ns, ntiles, rows = layout(nx, ny, nz)
    row = np.arange(nx * ny * nz, dtype=np.int64)
    i, jg, kg = row % nx, (row // nx) % ny, row // (nx * ny)
    J, jj, K, kk = jg // TJ, jg % TJ, kg // TK, kg % TK
    t = J + nJ * K
    lane = jj + TJ * kk
    frow = t * ns + (i + jj + kk)
    brow = t * ns + ((nx - 1 - i) + (TJ - 1 - jj) + (TK - 1 - kk))
    return frow, brow, lane


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_stage_two_writes_are_a_bijection_in_bounds(shape):
    nx, ny, nz = shape
    nJ, nK, ns, ntiles, rows = layout(nx, ny, nz)
    frow, brow, lane = stage2_slots(nx, ny, nz)
    for ne in (1, 2):
        r2 = frow * 3 * 64 + lane
        e0 = brow * ne * 64 + lane
        assert r2.min() >= 0 and r2.max() + 128 < rows * 3 * 64
        assert e0.min() >= 0 and e0.max() + 64 * (ne - 1) < rows * 2 * 64
    for r in (frow, brow):
        slot = r * 64 + lane
        assert np.unique(slot).size == slot.size  # one cell per slot
    # the faces the kernel fills: both sweeps' buffers, ntiles * ns * 60 each
    assert 2 * ntiles * ns * FACE == 2 * rows * FACE


def sweep_trace(nx, ny, nz, fwd):
    """Every (tile, step, lane) of one sweep: the cell handled (or -1) and the
    face reads and writes, as GridTile computes them."""
    nJ, nK, ns, ntiles, rows = layout(nx, ny, nz)
    t = np.arange(ntiles)[:, None, None]
    s = np.arange(ns + 2)[None, :, None]          # staged steps reach nst + 1 <= ns + 1
    lane = np.arange(64)[None, None, :]
    J, K = t % nJ, t // nJ
    jj, kk = lane & (TJ - 1), lane // TJ
    j, k = J * TJ + jj, K * TK + kk
    valid = (j < ny) & (k < nz)
    lag = jj + kk if fwd else (TJ - 1 - jj) + (TK - 1 - kk)
    i = s - lag if fwd else nx - 1 - (s - lag)
    active = valid & (i >= 0) & (i < nx) & (s < ns)
    cell = np.where(active, i + nx * (j + ny * k), -1)
    if fwd:
        pollJ = valid & (jj == 0) & (j > 0)
        pollK = valid & (kk == 0) & (k > 0)
        pubJ, pubK = valid & (jj == TJ - 1), valid & (kk == TK - 1)
        tJ, tK = t - 1, t - nJ
    else:
        pollJ = valid & (jj == TJ - 1) & (j + 1 < ny)
        pollK = valid & (kk == TK - 1) & (k + 1 < nz)
        pubJ, pubK = valid & (jj == 0), valid & (kk == 0)
        tJ, tK = t + 1, t + nJ
    b = np.broadcast_to
    shp = cell.shape
    return dict(nJ=nJ, ns=ns, ntiles=ntiles, rows=rows, t=b(t, shp), s=b(s, shp), lane=b(lane, shp),
                jj=b(jj, shp), kk=b(kk, shp), active=active, cell=cell, pollJ=b(pollJ, shp) & active,
                pollK=b(pollK, shp) & active, pubJ=b(pubJ, shp) & active, pubK=b(pubK, shp) & active,
                tJ=b(tJ, shp), tK=b(tK, shp))


@pytest.mark.parametrize("fwd", [True, False], ids=["forward", "backward"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_sweep_addresses_in_bounds_and_consistent(shape, fwd):
    nx, ny, nz = shape
    tr = sweep_trace(nx, ny, nz, fwd)
    ns, ntiles, rows, nJ = tr["ns"], tr["ntiles"], tr["rows"], tr["nJ"]
    nc = nx * ny * nz
    act, cell, t, s, lane = tr["active"], tr["cell"], tr["t"], tr["s"], tr["lane"]
    # every cell exactly once
    assert np.array_equal(np.sort(cell[act]), np.arange(nc))
    # the stage-two kernel's slot of the cell is the one this step reads
    frow, brow, slane = stage2_slots(nx, ny, nz)
    myrow = (t * ns + s)[act]
    assert np.array_equal((frow if fwd else brow)[cell[act]], myrow)
    assert np.array_equal(slane[cell[act]], lane[act])
    if fwd:  # y goes to the backward step of the same cell
        assert np.array_equal(brow[cell[act]], (t * ns + (ns - 1 - s))[act])
        yidx = ((t * ns + ns - 1) * 3 * 64 + lane - s * 3 * 64)[act]
        assert yidx.min() >= 0 and yidx.max() + 128 < rows * 3 * 64
    else:
        # z goes out in pairs of cells (c, c + 1) with c even, stored when
        # the sweep (i = nx - 1 down to 0) reaches c; the odd cell c + 1 was
        # the same lane's previous step, held until then.  Single cells at a
        # pencil's ends.
        i_of = cell % nx
        even = act & (cell % 2 == 0)
        pair = even & (i_of + 1 < nx)
        held = act & (cell % 2 == 1) & (i_of > 0)
        single = act & ~pair & ~held
        # a pair's partner is the lane's previous step, a held cell
        prev = np.full(cell.shape, -1)
        prev[:, 1:, :] = cell[:, :-1, :]
        assert np.array_equal(prev[pair], cell[pair] + 1)
        prev_held = np.zeros(cell.shape, dtype=bool)
        prev_held[:, 1:, :] = held[:, :-1, :]
        assert prev_held[pair].all()
        written = np.concatenate([cell[pair], cell[pair] + 1, cell[single]])
        # every cell's z written exactly once, in bounds
        assert np.array_equal(np.sort(written), np.arange(nc))
        assert (cell[pair] + 1).max(initial=0) < nc
    # staging: the matrix, right-hand side and e0 rows of steps 0 .. nst + 1
    H, R = CONFIGS[fwd]
    nst = (ns + 1) & ~1
    srow = t[:, :nst + 2, 0] * ns + np.minimum(s[:, :nst + 2, 0], ns - 1)
    NV = 27 if fwd else 36
    assert srow.min() >= 0 and (srow.max() + 1) * NV * 64 <= rows * NV * 64
    assert (srow.max() + 1) * 3 * 64 <= rows * 3 * 64 and (srow.max() + 1) * 2 * 64 <= rows * 2 * 64
    NR = 3 + (0 if fwd else 2)
    slot = (NV + NR + 6) * 64
    assert ((np.arange(nst + 2) % R).max() + 1) * slot <= R * slot
    # FP64 staging skips a load lane (two consecutive cell lanes of one tile
    # row, the same in every instruction) when neither cell is active at that
    # step: every cell the sweeping wave computes must still be staged
    m = np.arange(32)
    tt = np.arange(ntiles)[:, None, None]
    ss = np.arange(nst + 2)[None, :, None]
    on = np.zeros((ntiles, nst + 2, 32), dtype=bool)
    for u in (0, 1):
        c = 2 * m + u
        cjj, ckk = c % TJ, c // TJ
        cj, ck = (tt % nJ) * TJ + cjj, (tt // nJ) * TK + ckk
        lag = cjj + ckk if fwd else (TJ - 1 - cjj) + (TK - 1 - ckk)
        on |= (cj < ny) & (ck < nz) & (ss >= lag) & (ss < lag + nx)
    n = min(act.shape[1], nst + 2)
    assert not (act[:, :n, :] & ~np.repeat(on[:, :n, :], 2, axis=2)).any()
    # faces: published at (t, s), polled at (tJ, s + 15) / (tK, s + 3)
    nfaces = ntiles * ns * FACE
    def jface(tile, step, q, kk):
        return (tile * ns + step) * FACE + q * TK + kk
    def kface(tile, step, q, jj):
        return (tile * ns + step) * FACE + 3 * TK + q * TJ + jj
    pub = {}
    for name, m, f, sub in (("J", tr["pubJ"], jface, tr["kk"]), ("K", tr["pubK"], kface, tr["jj"])):
        if not m.any():
            pub[name] = {}
            continue
        idx = f(t[m], s[m], 2, sub[m])
        assert idx.min() >= 0 and idx.max() < nfaces
        pub[name] = dict(zip(f(t[m], s[m], 0, sub[m]).tolist(), cell[m].tolist()))
    for name, m, tn, skew, f, sub in (("J", tr["pollJ"], tr["tJ"], SKJ, jface, tr["kk"]),
                                      ("K", tr["pollK"], tr["tK"], SKK, kface, tr["jj"])):
        if not m.any():
            continue
        tt, ss = tn[m], s[m] + skew
        assert tt.min() >= 0 and tt.max() < ntiles and ss.max() < ns
        idx = f(tt, ss, 0, sub[m])
        assert idx.min() >= 0 and f(tt, ss, 2, sub[m]).max() < nfaces
        # the value read is the neighbour cell's, published by the neighbour tile
        got = np.array([pub[name][q] for q in idx.tolist()])
        c = cell[m]
        step = nx if name == "J" else nx * ny
        assert np.array_equal(got, c - step if fwd else c + step)


def test_backward_sweep_reads_no_e0_without_first_stage():
    """cptr_ilu_solve runs M2^-1 alone: the backward kernel gets e0t = null and
    must neither stage nor add e0 (the staging copy is guarded by e0t, the
    update by has_e0).  Checked on the kernel source, which is what the
    emulation above cannot see."""
    import os
    import re
    src = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "paper_2308_11892_amd", "csrc", "kernels.hip")).read()
    body = src[src.index("void k_ilu_grid("):src.index("// stage-two residual for the grid sweeps")]
    copies = re.findall(r".*wave_copy_to_lds<T, NE0 \* 64>\(e0t.*", body)
    assert copies and all("e0t)" in ln or "&& e0t" in ln for ln in copies), copies
    update = src[src.index("struct GridCell"):src.index("// The kernel: one workgroup per tile.")]
    assert "has_e0 = e0t != nullptr" in update and "has_e0 ? (double)r[3]" in update


def grid_pattern(nx, ny, nz):
    """The 7-point stencil in lexicographic order with sorted rows (what the
    library's grid check accepts), as CSR."""
    n = nx * ny * nz
    rp, ci = [0], []
    for c in range(n):
        x, y, z = c % nx, (c // nx) % ny, c // (nx * ny)
        cols = []
        if z > 0:
            cols.append(c - nx * ny)
        if y > 0:
            cols.append(c - nx)
        if x > 0:
            cols.append(c - 1)
        cols.append(c)
        if x < nx - 1:
            cols.append(c + 1)
        if y < ny - 1:
            cols.append(c + nx)
        if z < nz - 1:
            cols.append(c + nx * ny)
        ci += cols
        rp.append(len(ci))
    return np.array(rp), np.array(ci)


def diag_slot(nx, ny, r, d):
    """k_grid_ilu_diag's slot of column r + d within row r (mirrors its
    `slot` lambda)."""
    nxy = nx * ny
    xr, yr, zr = r % nx, (r // nx) % ny, r // nxy
    k = 0
    k += d > -nxy and zr > 0
    k += d > -nx and yr > 0
    k += d > -1 and xr > 0
    k += d > 0
    k += d > 1 and xr < nx - 1
    k += d > nx and yr < ny - 1
    return int(k)


@pytest.mark.parametrize("shape", [(2, 2, 2), (3, 2, 2), (7, 5, 3), (20, 20, 5), (16, 16, 8)],
                         ids=lambda s: "x".join(map(str, s)))
def test_grid_ilu_diag_slots_are_the_searched_ones(shape):
    """The factorisation kernel reads a neighbour's block at a slot computed
    from the cell's coordinates: for every cell and every neighbour it reads
    (its own diagonal, the lower blocks A_ck, and A_kc in each lower
    neighbour's row), that slot holds exactly that column, inside the row."""
    nx, ny, nz = shape
    rp, ci = grid_pattern(nx, ny, nz)
    nxy = nx * ny
    for c in range(nx * ny * nz):
        x, y, z = c % nx, (c // nx) % ny, c // nxy
        reads = [(c, 0)]
        for d, has in ((nxy, z > 0), (nx, y > 0), (1, x > 0)):
            if has:
                reads += [(c, -d), (c - d, d)]
        for r, d in reads:
            k = diag_slot(nx, ny, r, d)
            assert 0 <= k < rp[r + 1] - rp[r]
            assert ci[rp[r] + k] == r + d
