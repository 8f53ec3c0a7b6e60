"""Index arithmetic of the HIP kernels, emulated on the CPU (no GPU).

Mirrors the row partition the library builds (row blocks of at most
2048/C/cut_div arcs and 255 rows, rows above that row-split threshold split
into segments of 8192/C arcs, for the divisors 1, 2 and 4 the batch
autotuner races) and every
index formula of the step kernel, on CSRs in the library's internal vertex
order (stable by decreasing out-degree), and asserts that every load and
store lands inside its buffer -- including the empty trailing row blocks
that once read one entry past col_idx -- in both gather layouts: one 8-byte
value per (arc, column), and 32-bit inputs gathered as 8-byte column pairs
into blocks of twice the arcs.  For split scoring it emulates the
worklist that the member pushes fill and checks the capacity bound the host
allocates (entries past it would be dropped, not faulted, so a wrong bound
would give wrong results silently).
"""
import numpy as np
import pytest

from paper_1910_13874_amd import inputs

K_BLOCK, K_ROWS, K_SEG, K_LDS = 256, 255, 8192, 2048
WL_CHUNK = 512


def partition(rp, C, units=None, cut_div=1):
    """Row blocks and long-row segments for C columns gathered in `units`
    8-byte units per arc (C, or C/2 for column pairs)."""
    units = units or C
    n = len(rp) - 1
    nnz_blk = max(1, K_LDS // units // cut_div)
    seg_len = max(1, K_SEG // units)
    deg = np.diff(rp)
    blocks, segs, lrows = [], [], []
    r = 0
    while r < n:
        if deg[r] > nnz_blk:
            lrows.append(r)
            for j in range(int(rp[r]), int(rp[r + 1]), seg_len):
                segs.append((r, j, min(j + seg_len, int(rp[r + 1]))))
            r += 1
            continue
        r0, acc = r, 0
        while r < n and r - r0 < K_ROWS:
            d = deg[r]
            if d > nnz_blk or acc + d > nnz_blk:
                break
            acc += d
            r += 1
        blocks.append((r0, r, int(rp[r0]), int(rp[r])))
    return blocks, segs, lrows


def check_step(rp, ci, n, C, pairs=False, cut_div=1, hub=None):
    """pairs: 32-bit input gathered as column pairs (C >= 2): unit q of thread
    t loads elements u*C + 2k, +1 with k = unit mod C/2, staged as two 32-bit
    LDS slots; phase 2 reads slot j*C + c.  hub (with pairs, C >= 4): 16-bit
    level-2 counts gathered as 4-column units on the same partition, half
    as many units per thread: rows u < hub from the 32-bit table (elements
    u*C + 4k .. +3), every lane from the packed rows (elements (u - hub)*C +
    4k .. +3, row 0 for hub lanes), staged as four 32-bit LDS slots."""
    nnz = int(rp[-1])
    ci_alloc = max(1, nnz)
    if hub is not None:
        assert pairs and C >= 4 and 0 <= hub < n
        check_quads(rp, ci, n, C, cut_div, hub)
        return
    U = C // 2 if pairs else C
    blocks, segs, lrows = partition(rp, C, U, cut_div)
    cut = max(1, K_LDS // U // cut_div)
    deg = np.diff(rp)
    # every arc is in exactly one block or segment; long rows are those above the cut
    covered = sum(p1 - p0 for (_, _, p0, p1) in blocks) + sum(z - y for (_, y, z) in segs)
    assert covered == nnz
    assert all(deg[r] > cut for r in lrows)
    assert all(deg[r0:r1].max(initial=0) <= cut and p1 - p0 <= cut for (r0, r1, p0, p1) in blocks)
    PT = K_LDS // K_BLOCK
    RT = (K_ROWS + K_BLOCK) // K_BLOCK
    t = np.arange(K_BLOCK)
    mask_words = (n + 31) // 32 + 1
    for (r0, r1, p0, p1) in blocks:
        nrows, tot = r1 - r0, (p1 - p0) * U
        assert 1 <= nrows <= K_ROWS and 0 <= tot <= K_LDS
        jlo = p0 if tot > 0 else 0
        jmax = p1 - 1 if tot > 0 else 0
        for q in range(PT):  # col_idx loads, gathers, LDS stores
            j = np.minimum(jlo + (t + q * K_BLOCK) // U, jmax)
            assert j.min() >= 0 and j.max() < ci_alloc
            u = ci[j] if tot > 0 else np.zeros_like(j)
            assert u.min() >= 0 and u.max() < n
            if pairs:
                e = u * C + 2 * ((t + q * K_BLOCK) & (U - 1))
                assert e.min() >= 0 and (e + 1).max() < n * C and (e % 2 == 0).all()
            f = t + q * K_BLOCK
            slot = f[f < tot]  # staged only below the block's units
            assert slot.size == 0 or slot.max() < K_LDS
        if pairs and tot > 0:  # phase 2 reads 32-bit slot j*C + c of the staged arcs
            assert (p1 - p0 - 1) * C + C - 1 < 2 * tot
        for k in range(RT):  # row_ptr slice
            assert (r0 + np.minimum(t + k * K_BLOCK, nrows)).max() <= n
        nw = ((r0 + nrows - 1) >> 5) - (r0 >> 5) + 1
        assert ((r0 >> 5) + np.minimum(t, nw - 1)).max() < mask_words
        for k in range((K_ROWS + K_BLOCK - 1) // K_BLOCK):  # per-row masks
            rr = r0 + np.minimum(t + k * K_BLOCK, nrows - 1)
            assert rr.min() >= 0 and rr.max() < n
        # combining epilogue's early loads: row r0 + min((t/tpr)/C, nrows-1)
        tpr = min(K_BLOCK // C, 64)
        while tpr > 1 and nrows * C * tpr > K_BLOCK:
            tpr >>= 1
        rl0 = (t // tpr) // C
        assert (r0 + np.minimum(rl0, nrows - 1)).max() < n
        assert (p1 - p0) * U <= K_LDS
    for (r, y, z) in segs:  # long-row segments, 8 clamped loads per lane
        assert 0 <= y < z <= nnz and z - y <= max(1, K_SEG // U)
        lpc = K_BLOCK // U
        j0 = y + t // U
        while j0.min() < z:
            for q in range(8):
                jj = np.minimum(j0 + q * lpc, z - 1)
                assert jj.min() >= y and jj.max() < nnz
                if pairs:
                    e = ci[jj].astype(np.int64) * C + 2 * (t & (U - 1))
                    assert (e + 1).max() < n * C
            j0 = j0 + 8 * lpc


def check_quads(rp, ci, n, C, cut_div, hub, table_rows=None):
    """Index arithmetic of the 16-bit (IN_CNT16) gather on its own partition
    (C/4 eight-byte units per arc): row blocks stage every arc's packed
    8 bytes (elements u*C + 4k .. +3 of the packed rows, which cover every
    row) as 16-bit LDS values, loading rows below the cut from the 32-bit
    table (16 bytes at u*C + 4k), and the per-row sums fetch a marked
    value's 32-bit count at src*C + c, src read back from col_idx at the
    block's arc; long-row segments load the packed unit and, for hub rows
    or marked values, 16 bytes of the table (bucket blocks use the row
    blocks' formulas on the copied col_idx).  Also the byte extent of the layout against its
    allocation and the pushes' 32-bit words.  table_rows = n: the 16-bit copy
    of a stored level (cut 0), whose marked values any row may carry and
    whose 32-bit level holds every row."""
    nnz = int(rp[-1])
    GU = C // 4
    blocks, segs, _ = partition(rp, C, GU, cut_div)
    PT = K_LDS // K_BLOCK
    t = np.arange(K_BLOCK)
    pk_off = (hub * C * 4 + 255) // 256 * 256
    alloc = max(4 * n * C, pk_off + 2 * n * C)

    def packed(u, k):
        e16 = u * C + 4 * k
        assert e16.min() >= 0 and (e16 + 3).max() < n * C and (e16 % 4 == 0).all()
        assert pk_off + 2 * ((e16 + 3).max() + 1) <= alloc

    rows32 = hub if table_rows is None else table_rows

    def table(u, k_or_c, width):
        hb = u < rows32
        if hb.any():
            e32 = u[hb] * C + k_or_c[hb] if np.ndim(k_or_c) else u[hb] * C + k_or_c
            assert e32.min() >= 0 and (e32 + width - 1).max() < rows32 * C

    for (r0, r1, p0, p1) in blocks:
        tot = (p1 - p0) * GU
        assert tot <= K_LDS
        jlo = p0 if tot > 0 else 0
        jmax = p1 - 1 if tot > 0 else 0
        for q in range(PT):
            f = t + q * K_BLOCK
            j = np.minimum(jlo + f // GU, jmax)
            assert j.min() >= 0 and j.max() < max(1, nnz)
            u = ci[j] if tot > 0 else np.zeros_like(j)
            packed(u, f & (GU - 1))
            table(u, 4 * (f & (GU - 1)), 4)  # rows below the cut: their 32-bit counts
            slot = f[f < tot]  # 8-byte slots of four 16-bit values
            assert slot.size == 0 or 4 * slot.max() + 3 < 4 * K_LDS
        if tot > 0:  # phase 2: 16-bit slot j*C + c; hub rows from the table
            assert (p1 - p0 - 1) * C + C - 1 < 4 * tot
            src = ci[p0:p1]
            for c in (0, C - 1):
                table(src, c, 1)
    for (r, y, z) in segs:
        lpu = K_BLOCK // GU
        j0 = y + t // GU
        while j0.min() < z:
            for q in range(8):
                jj = np.minimum(j0 + q * lpu, z - 1)
                assert jj.min() >= y and jj.max() < nnz
                u = ci[jj].astype(np.int64)
                packed(u, t & (GU - 1))
                table(u, 4 * (t & (GU - 1)), 4)
            j0 = j0 + 8 * lpu
    # the pushes' 32-bit words of packed entries (v >= hub, any column)
    o = (n - 1) * C + (C - 1)
    assert pk_off + 2 * (o & ~1) + 4 <= alloc


def internal_csr(g):
    """The library's storage: vertices by decreasing out-degree (stable),
    rows = in-neighbours, sorted."""
    n = g.n
    rows = np.repeat(np.arange(n), np.diff(g.row_ptr))
    outdeg = np.bincount(g.col_idx, minlength=n)
    order = np.argsort(-outdeg, kind="stable")
    new = np.empty(n, np.int64)
    new[order] = np.arange(n)
    v, u = new[rows], new[g.col_idx]
    idx = np.lexsort((u, v))
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, v + 1, 1)
    return np.cumsum(rp), u[idx].astype(np.int64)


def graphs():
    r = inputs.uniform_ints(2 * 9000, 2000, 61)
    return [
        inputs.from_edges(5, [], [], name="edgeless"),
        inputs.erdos_renyi(3000, 2000, 7),       # many isolated vertices
        inputs.erdos_renyi(1000, 5000, 1),
        inputs.barabasi_albert(20000, 5, 2),
        inputs.rmat(14, 16, seed=18),
        inputs.from_edges(2, [0], [1], name="K2"),
        inputs.from_edges(9000, np.zeros(8999, np.int32), np.arange(1, 9000, dtype=np.int32),
                          name="star"),           # one row longer than any block
        inputs.from_edges(2000, r[0::2], r[1::2], symmetrize=False, name="dir"),
    ]


@pytest.mark.parametrize("g", graphs(), ids=lambda g: g.name or str(g.n))
def test_step_indices_in_bounds(g):
    for rp, ci in ((np.asarray(g.row_ptr, np.int64), np.asarray(g.col_idx, np.int64)),
                   internal_csr(g)):
        for C in (1, 2, 4, 8, 16, 32, 64):
            for cut_div in ((1, 2, 4) if C in (1, 2, 16, 64) else (1,)):
                check_step(rp, ci, g.n, C, cut_div=cut_div)
                if C >= 2:
                    check_step(rp, ci, g.n, C, pairs=True, cut_div=cut_div)
                if C in (4, 8, 32):  # 16-bit gathers: one and two units per arc, and 8
                    for hub in sorted({0, g.n // 8, g.n - 1}):
                        check_quads(rp, ci, g.n, C, cut_div, hub)
                    check_quads(rp, ci, g.n, C, cut_div, 0, table_rows=g.n)


K_HUB_ROWS, K_HUB_SHARE_DIV = 2048, 10


def hub_copy_rows(g, rp):
    """Rows of the LDS copy in single-column count steps, as graph creation
    sets them: the first kHubRows internal rows (kHubRows or n) when they are
    the sources of at least 1/kHubShareDiv of the arcs of an undirected
    unweighted graph, else 0."""
    h = min(K_HUB_ROWS, g.n)
    nnz = int(rp[-1])
    if g.directed or nnz == 0 or int(rp[h]) * K_HUB_SHARE_DIV < nnz:
        return 0
    return h


@pytest.mark.parametrize("g", graphs(), ids=lambda g: g.name or str(g.n))
def test_hub_copy_indices(g):
    """The copy's loads (clamped rows, also when it is off), its LDS slots and
    the reads of gathered sources stay in bounds; R-MAT takes the copy (on
    BA n=20,000 too: its 2,048 rows are a tenth of the vertices)."""
    rp, ci = internal_csr(g)
    hc = hub_copy_rows(g, rp)
    assert 0 <= hc <= min(K_HUB_ROWS, g.n)
    t = np.arange(K_BLOCK)
    for q in range(K_HUB_ROWS // K_BLOCK):
        rows = np.minimum(t + q * K_BLOCK, max(hc - 1, 0))
        assert rows.max() < g.n
        assert (t + q * K_BLOCK).max() < K_HUB_ROWS  # LDS slot
    if ci.size:
        src = ci
        assert np.minimum(src, K_HUB_ROWS - 1).max() < K_HUB_ROWS
        assert (src[src < hc] < g.n).all()
    if g.name and g.name.startswith("rmat"):
        assert hc == K_HUB_ROWS


def wl_need(n, nnz, deg_sum):
    return min(n, deg_sum) + nnz // WL_CHUNK + 1


@pytest.mark.parametrize("name", ["ba", "star", "rmat"])
def test_split_worklist_fits_capacity(name):
    """Emulate the member pushes of a tile: a non-member neighbour y claimed
    first adds ceil(deg(y)/512) entries (y, column, chunk); the total must fit
    the capacity the host computes from the members' degree sums, and every
    entry's chunk must start inside row y and fit the 24-bit field."""
    if name == "ba":
        g = inputs.barabasi_albert(5000, 4, 3)
    elif name == "star":
        g = inputs.from_edges(9000, np.zeros(8999, np.int32), np.arange(1, 9000, dtype=np.int32))
    else:
        g = inputs.rmat(13, 16, seed=9)
    rp, ci = internal_csr(g)
    n, nnz = g.n, int(rp[-1])
    deg = np.diff(rp)
    rng = np.random.default_rng(5)
    for C in (1, 8, 16):
        groups = [np.unique(rng.integers(0, n, int(rng.integers(1, 300)))) for _ in range(C)]
        if name == "star":
            groups[0] = np.array([1])  # a leaf: its neighbour is the hub (8999 arcs)
        entries, cap = 0, 0
        for S in groups:
            member = np.zeros(n, bool)
            member[S] = True
            claimed = set()
            for s in S:
                for y in ci[rp[s]:rp[s + 1]]:
                    if not member[y] and y not in claimed:
                        claimed.add(int(y))
                        chunks = (int(deg[y]) + WL_CHUNK - 1) // WL_CHUNK
                        for q in range(chunks):
                            assert q < (1 << 24) and rp[y] + q * WL_CHUNK < rp[y + 1]
                        entries += chunks
            cap += wl_need(n, nnz, int(deg[S].sum()))
        assert entries <= cap, (name, C, entries, cap)


def check_plan_matches_emulation(ged, rp, ci, n, U, cut_div):
    """Without buckets the library's own planner gives exactly the partition
    emulated above."""
    pl = ged.partition_plan(rp, ci, n, U, cut_div, 0)
    blocks, segs, lrows = partition(rp, U, U, cut_div)
    assert pl["bucketed"] == 0 and pl["cut"] == max(1, K_LDS // U // cut_div)
    assert [tuple(b) for b in pl["blocks"]] == [tuple(map(int, b)) for b in blocks]
    assert [tuple(s[:3]) for s in pl["grid2"]] == [tuple(map(int, s)) for s in segs]
    assert list(pl["long_rows"]) == list(lrows)
    assert pl["n_segs"] == pl["n_grid2"] == len(segs)


def check_buckets(ged, rp, ci, n, C, pairs, cut_div, bucket_rows, rng):
    """Source-bucketed plan from the library's planner: every long row's arcs
    are split into pieces inside one bucket, copied, and summed back exactly
    by the fix-up's piece lists; bucket blocks respect the block limits and
    are dealt to the XCDs (grid position n_blocks + i runs on XCD
    (n_blocks + i) mod 8) in eight contiguous runs; and every index the step
    kernel's bucket blocks and the fix-up form stays inside its buffer.
    pairs == "quad": 16-bit inputs, C/4 four-column units per arc (staged
    as four 16-bit values; the packed rows cover every vertex)."""
    quad = pairs == "quad"
    U = C // 4 if quad else C // 2 if pairs else C
    pl = ged.partition_plan(rp, ci, n, U, cut_div, bucket_rows)
    cut = pl["cut"]
    deg = np.diff(rp)
    lrows = pl["long_rows"]
    if len(lrows) == 0:
        assert pl["bucketed"] == 0
        return
    assert pl["bucketed"] == 1 and pl["bucket_rows"] == bucket_rows
    nseg, bk_ptr, bk_ci, lsub = pl["n_segs"], pl["bk_ptr"], pl["bk_ci"], pl["bk_lsub"]
    lf = pl["long_first"]
    assert bk_ptr[0] == 0 and np.all(np.diff(bk_ptr) >= 1) and bk_ptr[-1] == pl["bk_arcs"]
    assert np.all(np.diff(bk_ptr) <= cut)
    assert pl["bk_arcs"] == int(deg[lrows].sum())
    # pieces of each row: its arcs in order, each piece inside one bucket
    assert lf[0] == 0 and np.all(np.diff(lf) >= 1) and lf[-1] == nseg
    assert sorted(lsub.tolist()) == list(range(nseg))
    bucket_of_piece = np.empty(nseg, np.int64)
    for l, r in enumerate(lrows):
        pieces = [bk_ci[bk_ptr[s]:bk_ptr[s + 1]] for s in lsub[lf[l]:lf[l + 1]]]
        assert np.array_equal(np.concatenate(pieces), ci[rp[r]:rp[r + 1]])
        for s, p in zip(lsub[lf[l]:lf[l + 1]], pieces):
            b = p // bucket_rows
            assert (b == b[0]).all()
            bucket_of_piece[s] = b[0]
    assert np.all(np.diff(bucket_of_piece) >= 0)  # pieces numbered bucket by bucket
    # exact sums through the pieces and the fix-up lists
    x = rng.integers(0, 1000, n).astype(np.int64)
    piece_sum = np.array([x[bk_ci[bk_ptr[s]:bk_ptr[s + 1]]].sum() for s in range(nseg)])
    for l, r in enumerate(lrows):
        assert piece_sum[lsub[lf[l]:lf[l + 1]]].sum() == x[ci[rp[r]:rp[r + 1]]].sum()
    # bucket blocks: limits, cover, XCD runs
    g2 = pl["grid2"]
    nb, n_blocks = len(g2), pl["n_blocks"]
    assert pl["n_grid2"] == nb
    order = sorted(range(nb), key=lambda i: g2[i][0])
    assert [int(g2[i][0]) for i in order] == [0] + [int(g2[i][1]) for i in order[:-1]]
    assert int(g2[order[-1]][1]) == nseg
    runs = [[i for i in range(nb) if (n_blocks + i) % 8 == xcd] for xcd in range(8)]
    seq = [int(g2[i][0]) for xcd in range(8) for i in runs[xcd]]
    assert seq == sorted(seq)  # XCD 0's run first, each run in piece order
    PT = K_LDS // K_BLOCK
    RT = (K_ROWS + K_BLOCK) // K_BLOCK
    t = np.arange(K_BLOCK)
    for (s0, s1, a0, a1) in g2:
        npc, tot = s1 - s0, (a1 - a0) * U
        assert 1 <= npc <= K_ROWS and U <= tot <= K_LDS
        assert bk_ptr[s0] == a0 and bk_ptr[s1] == a1
        for q in range(PT):
            j = np.minimum(a0 + (t + q * K_BLOCK) // U, a1 - 1)
            assert j.min() >= 0 and j.max() < len(bk_ci)
            u = bk_ci[j]
            assert u.min() >= 0 and u.max() < n
            if quad:
                e = u.astype(np.int64) * C + 4 * ((t + q * K_BLOCK) & (U - 1))
                assert (e + 3).max() < n * C
            elif pairs:
                e = u.astype(np.int64) * C + 2 * ((t + q * K_BLOCK) & (U - 1))
                assert (e + 1).max() < n * C
            f = t + q * K_BLOCK
            assert f[f < tot].max(initial=0) < K_LDS
        for k in range(RT):
            assert (s0 + np.minimum(t + k * K_BLOCK, npc)).max() <= nseg
        # phase 2: arc slots j*C + c of the staged values, piece sums to seg_out
        assert (a1 - a0) * C <= (4 if quad else 2 if pairs else 1) * K_LDS
        assert s1 <= nseg
    # fix-up: entries of the piece lists name seg_out slots
    assert lsub.max() < nseg and lf.max() <= len(lsub)


@pytest.mark.parametrize("g", graphs(), ids=lambda g: g.name or str(g.n))
def test_bucket_plan_in_bounds(g):
    from paper_1910_13874_amd import ged
    rng = np.random.default_rng(5)
    rp, ci = internal_csr(g)
    for U, cut_div in ((1, 1), (2, 1), (4, 1), (4, 2), (8, 4), (32, 1)):
        check_plan_matches_emulation(ged, rp, ci, g.n, U, cut_div)
    for C, pairs in ((1, False), (2, False), (4, False), (2, True), (4, True), (8, True),
                     (4, "quad"), (8, "quad")):
        for cut_div in (1, 2, 4):
            for br in (1, 7, 64, 4096, 1 << 20):
                check_buckets(ged, rp, ci, g.n, C, pairs, cut_div, br, rng)
