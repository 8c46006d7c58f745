"""The strip kernels' work decomposition, modelled on the CPU.

A Python restatement of the index arithmetic of every strip-shaped kernel that
is built -- the single-step strip (k_step_strip), the fused periodic kernels
(k_step_fused, K = 2 and 3), the fused kernel with walls (k_step_fused_wall),
the multiphase strips (k_step_sc_strip, k_step_sc_fused), the batched kernel
(k_step_batch over its flattened item lists) and the 3-D lane-exchange tiles
(k_step3_lane) -- checks, for many shapes and
every launch configuration, that

  * every moment load lies inside the parity block it reads,
  * every flag load (a pack of VEC bytes) lies inside the flag plane,
  * every store lies inside the parity block it writes or inside its 1 KiB
    region of the grid's 3 KiB trash area,
  * a stored chunk never crosses the row pitch (padded last chunks stay in the
    row padding), and
  * every (field, row, chunk) of the grid is written exactly once.

It also checks the trash bound 64 * VEC * sizeof(S) <= 1024 for every (storage,
columns per lane) pair the kernel table builds.  It needs no GPU; it guards the
decomposition, not the arithmetic.
"""
import numpy as np
import pytest

TRASH_REGION = 1024


def layout(nx, ny, c, snapshot=True):
    """The row-interleaved layout of the runtime: [parity][ny][3][pitch], flags, a
    snapshot, the reduction workspace and the trash area."""
    ru = lambda v, a: (v + a - 1) // a * a
    pitch = ru(nx, 64)
    rs = 3 * pitch
    field_off = [q * pitch * c for q in range(3)]
    state = ru(3 * pitch * ny * c, 256)
    flags_off = 2 * state
    flags_bytes = ru(pitch * ny, 256)
    off = flags_off + flags_bytes + (state if snapshot else 0)
    off += ru(1024 * 6 * 8, 256) + 256
    trash_off = off
    off += 3 * TRASH_REGION
    return dict(pitch=pitch, rs=rs, field_off=field_off, state=state, flags_off=flags_off,
                flags_bytes=flags_bytes, trash_off=trash_off, total=off)


# Per kernel: rows a strip loads beyond its NY stored rows (half above, half
# below), whether the last chunk of a row may be padded (only kernels that run
# on grids not periodic in x), and whether it loads flags.
KERNELS = {
    "strip": dict(halo=lambda K: 1, padded=True, flags=None),      # flags when the grid has walls
    "fused": dict(halo=lambda K: K, padded=False, flags=False),
    "fused_wall": dict(halo=lambda K: 2, padded=True, flags=True),
    "sc_strip": dict(halo=lambda K: 2, padded=False, flags=False),
    "sc_fused": dict(halo=lambda K: 4, padded=False, flags=False),
    "batch": dict(halo=lambda K: 1, padded=True, flags=True),
}


def wrap_axis(c, n, periodic):
    """Vectorised wrap_axis of the device code: wrapped when periodic (any
    distance), -1 outside a non-periodic axis."""
    c = np.asarray(c)
    out = np.where((c >= 0) & (c < n), c, np.mod(c, n) if periodic else -1)
    return out


def strip_accesses(kind, L, nx, ny, c, VEC, NY, K, chunk0, y0, px, py, haswall, written, trash_base):
    """Every load and store of one wavefront's strip, checked; stores counted."""
    spec = KERNELS[kind]
    halo = spec["halo"](K)
    NR = NY + 2 * halo
    lane = np.arange(64)
    nch = -(-nx // VEC) if spec["padded"] else nx // VEC
    ch = chunk0 - 1 + lane
    inside = (ch >= 0) & (ch < nch)
    if spec["padded"] and not px:
        col_ok = inside
        chw = np.where(inside, ch, 0)
    else:
        col_ok = np.ones(64, bool)
        chw = np.where(inside, ch, np.mod(ch, nch))
    xc = np.where(col_ok, chw * VEC, 0)
    lane_out = (lane >= 1) & (lane <= 62) & (ch < nch)
    assert (xc + VEC <= L["pitch"]).all()
    loads_flags = spec["flags"] if spec["flags"] is not None else haswall
    periodic_rows = py if spec["padded"] else True
    for p_src in (0, 1):
        src = p_src * L["state"]
        dst = (1 - p_src) * L["state"]
        for i in range(NR):
            rr = int(wrap_axis(y0 - halo + i, ny, periodic_rows))
            row = rr if rr >= 0 else 0
            assert 0 <= row < ny
            for q in range(3):
                lo = src + L["field_off"][q] + (row * L["rs"] + xc) * c
                assert (lo >= src).all() and (lo + VEC * c <= src + L["state"]).all()
            if loads_flags:
                lo = L["flags_off"] + row * L["pitch"] + xc
                assert (lo >= L["flags_off"]).all()
                assert (lo + VEC <= L["flags_off"] + L["flags_bytes"]).all()
            if i < NR - NY:
                continue
            t = y0 + i - (NR - NY)
            ok = (t < ny) & lane_out
            for q in range(3):
                lo_ok = dst + L["field_off"][q] + (t * L["rs"] + xc) * c
                lo_tr = L["trash_off"] + q * TRASH_REGION + lane * VEC * c
                assert (lo_tr + VEC * c <= L["trash_off"] + (q + 1) * TRASH_REGION).all()
                assert (lo_tr + VEC * c <= L["total"]).all()
                if ok.any():
                    assert (lo_ok[ok] >= dst).all() and (lo_ok[ok] + VEC * c <= dst + L["state"]).all()
                if p_src == 0:
                    for cc in ch[ok]:
                        key = (q, t, int(cc))
                        written[key] = written.get(key, 0) + 1


def launch_strips(nch, ny, NY, waves, cus=256):
    """The strips of one launch in the order the blocks, XCD ranges and waves of
    the kernel visit them: (chunk0, y0) pairs."""
    strips_x = (nch + 61) // 62
    strips_y = (ny + NY - 1) // NY
    units = (strips_x * strips_y + 3) // 4
    if waves > 0:
        blocks = min(max(8, (cus * waves // 4) // 8 * 8), (units + 7) // 8 * 8)
    else:
        blocks = (units + 7) // 8 * 8
    per_xcd = (units + 7) // 8
    out = []
    for b in range(blocks):
        xcd, local = b & 7, b >> 3
        begin, end = xcd * per_xcd, min(units, xcd * per_xcd + per_xcd)
        stride = blocks >> 3 if waves > 0 else units
        u = begin + local
        while u < end:
            for wave in range(4):
                s = u * 4 + wave
                sy, sx = divmod(s, strips_x)
                if sy < strips_y:
                    out.append((sx * 62, sy * NY))
            u += stride
    return out


def check_kernel(kind, nx, ny, c, VEC, NY, K, waves, periodic, haswall=True):
    L = layout(nx, ny, c)
    px, py = bool(periodic & 1), bool(periodic & 2)
    nch = -(-nx // VEC) if KERNELS[kind]["padded"] else nx // VEC
    written = {}
    for chunk0, y0 in launch_strips(nch, ny, NY, waves):
        strip_accesses(kind, L, nx, ny, c, VEC, NY, K, chunk0, y0, px, py, haswall, written, None)
    assert len(written) == 3 * ny * nch, (kind, nx, ny, VEC, NY, waves)
    assert set(written.values()) == {1}


SHAPES = [(512, 77, 0), (512, 77, 3), (264, 61, 0), (264, 61, 1), (264, 61, 2), (17, 9, 3),
          (3, 3, 3), (3, 3, 0), (64, 32, 1), (124, 30, 3), (130, 5, 2), (131, 45, 0), (517, 33, 2),
          (250, 20, 0), (255, 255, 0), (33, 70, 0), (1000, 7, 3)]

# The built (storage bytes, columns per lane) pairs of each kernel family, with the
# strip heights and steps per launch it is built for.
BUILT = {
    "strip": [((8, 1), (6, 14), 1), ((8, 2), (6, 14), 1), ((4, 1), (6, 14), 1), ((4, 2), (6, 14), 1),
              ((4, 4), (6, 14), 1), ((2, 1), (6, 14), 1), ((2, 2), (6, 14), 1), ((2, 4), (6, 14), 1),
              ((2, 8), (6, 14), 1)],
    "fused": [((4, 4), (6, 14, 22, 28), 3), ((4, 4), (6, 14, 22, 28), 2), ((8, 2), (6, 14), 2),
              ((4, 2), (6, 14), 2), ((2, 2), (6, 14, 22, 30), 2), ((2, 4), (6, 14), 2)],
    "fused_wall": [((8, 2), (2, 6, 14), 2), ((4, 2), (2, 6, 14, 30), 2), ((2, 2), (2, 6, 14, 30), 2)],
    "sc_strip": [((8, 2), (6, 14), 1), ((4, 2), (6, 14), 1), ((4, 4), (6, 14), 1), ((2, 2), (6, 14), 1)],
    "sc_fused": [((4, 4), (6, 14, 22), 2)],
    "batch": [((8, 1), (6, 14), 1), ((8, 2), (6, 14), 1), ((4, 1), (6, 14), 1), ((4, 2), (6, 14), 1),
              ((4, 4), (6, 14), 1), ((2, 1), (6, 14), 1), ((2, 2), (6, 14), 1), ((2, 4), (6, 14), 1)],
}


@pytest.mark.parametrize("kind", sorted(BUILT))
def test_trash_area_holds_a_wavefront_of_every_built_pair(kind):
    """Lane l stores VEC values at trash + l * VEC + q * 1024 / sizeof(S): the 64
    lanes fill at most one 1 KiB region per field."""
    for (c, vec), _, _ in BUILT[kind]:
        assert 64 * vec * c <= TRASH_REGION, (kind, c, vec)


def _fits(kind, nx, periodic, vec):
    if KERNELS[kind]["padded"]:
        return nx % vec == 0 or not periodic & 1
    return nx % vec == 0


@pytest.mark.parametrize("nx,ny,periodic", SHAPES)
@pytest.mark.parametrize("kind", ["strip", "fused_wall"])
def test_walled_kernels_in_bounds_and_write_once(kind, nx, ny, periodic):
    for (c, vec), rows, K in BUILT[kind]:
        if not _fits(kind, nx, periodic, vec):
            continue
        for NY in rows:
            for waves in (0, 8):
                check_kernel(kind, nx, ny, c, vec, NY, K, waves, periodic, haswall=True)


@pytest.mark.parametrize("nx,ny", [(s[0], s[1]) for s in SHAPES if s[2] == 3])
@pytest.mark.parametrize("kind", ["fused", "sc_strip", "sc_fused", "strip"])
def test_periodic_kernels_in_bounds_and_write_once(kind, nx, ny):
    for (c, vec), rows, K in BUILT[kind]:
        if nx % vec:
            continue
        for NY in rows:
            for waves in (0, 8):
                check_kernel(kind, nx, ny, c, vec, NY, K, waves, 3, haswall=False)


def test_the_faulted_case_shape_is_in_bounds():
    """The 512 x 77 cavity (not periodic) in binary16 storage at 1, 2 and 4 columns per
    lane, 6 and 14 rows, one wavefront per strip and 8 per CU, as the kernel-family
    test runs it."""
    for vec in (1, 2, 4):
        for NY in (6, 14):
            for waves in (0, 8):
                check_kernel("strip", 512, 77, 2, vec, NY, 1, waves, 0, haswall=True)


def _vec_class(prec_bytes, nx, px):
    """Columns per lane of a grid in a batch: the widest of 1, 2, 4 (1, 2 in FP64) that
    divides nx or whose last chunk may be padded, and no wider than the grid."""
    for v in ((2, 1) if prec_bytes == 8 else (4, 2, 1)):
        if (nx % v == 0 or not px) and 64 * v <= max(64, nx):
            return v
    return 1


@pytest.mark.parametrize("c", [8, 4, 2])
def test_batch_item_lists_in_bounds_and_write_once(c):
    """A batch of uneven grids: the items (slot, strip) of each class, the grid-stride
    loop of k_step_batch over them, every grid's accesses inside its own allocation."""
    rng = np.random.default_rng(4)
    sizes = [(int(n), int(m), int(p)) for n, m, p in zip(rng.integers(3, 300, 14), rng.integers(3, 200, 14),
                                                        rng.integers(0, 4, 14))]
    sizes += [(32, 32, 0), (131, 45, 0), (256, 3, 1), (3, 3, 3)]
    grids = []
    for nx, ny, per in sizes:
        vec = _vec_class(c, nx, per & 1)
        grids.append(dict(nx=nx, ny=ny, per=per, vec=vec, L=layout(nx, ny, c), written={}))
    for rows in (6, 14):
        for blocks in (1, 7, 512):
            for cls in sorted({g["vec"] for g in grids}):
                items = []
                for slot, g in enumerate(grids):
                    if g["vec"] != cls:
                        continue
                    nch = -(-g["nx"] // cls)
                    sx = (nch + 61) // 62
                    sy = (g["ny"] + rows - 1) // rows
                    # (slot, 4 * strip + kind), any kind
                    items += [(slot, (k << 2) | (k % 3)) for k in range(sx * sy)]
                visited = []
                for b in range(blocks):
                    for wave in range(4):
                        it = b * 4 + wave
                        while it < len(items):
                            visited.append(items[it])
                            it += blocks * 4
                assert sorted(visited) == sorted(items)
                for slot, y in visited:
                    k = y >> 2
                    g = grids[slot]
                    nch = -(-g["nx"] // cls)
                    strips_x = (nch + 61) // 62
                    sy, sx = divmod(k, strips_x)
                    strip_accesses("batch", g["L"], g["nx"], g["ny"], c, cls, rows, 1, sx * 62, sy * rows,
                                   bool(g["per"] & 1), bool(g["per"] & 2), True, g["written"], None)
            for g in grids:
                nch = -(-g["nx"] // g["vec"])
                assert len(g["written"]) == 3 * g["ny"] * nch
                assert set(g["written"].values()) == {1}
                g["written"] = {}


def strip_interior(flags, per, VEC, chunk0, y0, NY, HALO):
    """Model of strip_interior: the stored chunks widened by HALO columns and the
    strip's rows widened by HALO rows, all inside the grid and FLUID."""
    ny, nx = flags.shape
    nch = -(-nx // VEC)
    ce = min(nch, chunk0 + 62)
    if chunk0 < 1 or ce <= chunk0 or ce * VEC + HALO > nx or y0 < HALO or y0 + NY + HALO > ny:
        return False
    any_ = 0
    for lane in range(64):
        ch = chunk0 - 1 + lane
        lo = VEC - HALO if ch == chunk0 - 1 else 0
        hi = HALO if ch == ce else (VEC if ch < ce else 0)
        for i in range(NY + 2 * HALO):
            for v in range(lo, hi):
                any_ |= int(flags[y0 - HALO + i, ch * VEC + v])   # inside: ch * VEC + v < nx
    return any_ == 0


def strip_colwall(flags, per, VEC, chunk0, y0, NY, HALO):
    """Model of strip_colwall: the flags of the 64 lanes' chunks, as the wall-aware
    body loads them, equal in every footprint row of each column."""
    ny, nx = flags.shape
    px, py = bool(per & 1), bool(per & 2)
    if not py and (y0 < HALO or y0 + NY + HALO > ny):
        return False
    padded = np.full((ny, -(-nx // VEC) * VEC), 1, np.uint8)   # row padding is SOLID
    padded[:, :nx] = flags
    nch = padded.shape[1] // VEC
    for lane in range(64):
        ch = chunk0 - 1 + lane
        if ch < 0 or ch >= nch:
            if not px:
                continue
            ch %= nch
        rows = [int(wrap_axis(y0 - HALO + i, ny, py)) for i in range(NY + 2 * HALO)]
        cols = padded[rows, ch * VEC:(ch + 1) * VEC]
        if (cols != cols[0]).any():
            return False
    return True


@pytest.mark.parametrize("VEC,HALO", [(1, 1), (2, 1), (4, 1), (2, 2)])
def test_strip_kinds_hold_what_their_bodies_assume(VEC, HALO):
    """Brute force over cavities, channels and obstacle fields: a strip classed
    interior has every node within HALO of a stored node inside the grid and FLUID;
    a strip classed column-walls sees the same flags in every row of each column."""
    from paper_1912_09327_amd import inputs as I
    rng = np.random.default_rng(11)
    geos = []
    for L in (37, 70, 130, 261, 300):
        f = I.cavity(L, 0.05)[0]
        geos.append((f, 0))
        ch, per = I.channel(L, L // 2 + 3)
        geos.append((ch, per))
    geos.append((I.cavity(600, 0.05, ny=40)[0], 0))
    geos.append(I.channel(600, 40))
    f = np.zeros((50, 140), np.uint8)
    f[rng.random(f.shape) < 0.02] = I.SOLID
    geos += [(f, 3), (f, 0)]
    seen = {"interior": 0, "colwall": 0}
    for flags, per in geos:
        ny, nx = flags.shape
        nch = -(-nx // VEC)
        for NY in (2, 6, 14):
            for sy in range(-(-ny // NY)):
                for sx in range(-(-nch // 62)):
                    c0, y0 = sx * 62, sy * NY
                    if strip_interior(flags, per, VEC, c0, y0, NY, HALO):
                        seen["interior"] += 1
                        ce = min(nch, c0 + 62)
                        xs = [x for x in range(c0 * VEC, ce * VEC) if x < nx]
                        ys = [y for y in range(y0, min(y0 + NY, ny))]
                        for y in ys:
                            for x in xs:
                                for dy in range(-HALO, HALO + 1):
                                    for dx in range(-HALO, HALO + 1):
                                        assert 0 <= y + dy < ny and 0 <= x + dx < nx
                                        assert flags[y + dy, x + dx] == I.FLUID
                    elif strip_colwall(flags, per, VEC, c0, y0, NY, HALO):
                        seen["colwall"] += 1
    assert seen["interior"] > 0 and seen["colwall"] > 0


@pytest.mark.parametrize("VEC", [2, 4])
def test_interior_strips_of_walled_grids_stay_inside_without_wrapping(VEC):
    """The walled two-step kernels hand interior strips (strip_interior, two steps)
    to the wall-free body, which wraps chunks and rows as on a periodic grid and
    takes nch = nx // VEC.  For such a strip every chunk its 64 lanes load and every
    row it walks (NY + 4) lies inside the grid, so nothing wraps, and every stored
    chunk lies below nx // VEC."""
    from paper_1912_09327_amd import inputs as I
    rng = np.random.default_rng(12)
    geos = [I.cavity(L, 0.05)[0] for L in (61, 130, 263, 301, 517)]
    geos.append(I.cavity(600, 0.05, ny=70)[0])
    f = np.zeros((60, 530), np.uint8)
    f[rng.random(f.shape) < 0.01] = I.SOLID
    geos.append(f)
    seen = 0
    for flags in geos:
        ny, nx = flags.shape
        nch_ceil, nch_floor = -(-nx // VEC), nx // VEC
        for NY in (2, 6, 14, 30):
            for sy in range(-(-ny // NY)):
                for sx in range(-(-nch_ceil // 62)):
                    c0, y0 = sx * 62, sy * NY
                    if not strip_interior(flags, 0, VEC, c0, y0, NY, 2):
                        continue
                    seen += 1
                    ch = c0 - 1 + np.arange(64)
                    assert (ch >= 0).all() and (ch < nch_floor).all()
                    rows = y0 - 2 + np.arange(NY + 4)
                    assert (rows >= 0).all() and (rows < ny).all()
                    stored = ch[1:63]
                    assert (stored[stored < nch_floor] == stored).all()
    assert seen > 0


@pytest.mark.parametrize("nx,ny,nz,zc", [(70, 21, 9, 32), (64, 4, 16, 32), (130, 7, 20, 16), (5, 3, 1, 32),
                                         (124, 9, 40, 32), (62, 8, 33, 16), (512, 512, 64, 32)])
def test_3d_lane_tiles_write_every_node_once(nx, ny, nz, zc):
    """k_step3_lane (fully periodic 3-D grids): tiles of 62 target columns, 8 rows and
    zc planes, one block of 8 wavefronts each, launched as the tile count rounded up to
    a multiple of 8 blocks, block b taking tile (b % 8) * per + b // 8.  Lane l of the
    wavefront of row y0 + w holds column x0 - 1 + l (lanes 1 to 62 are targets, lanes
    0 and 63 halo columns).  Every tile is taken once, every load (own row, the halo
    rows y0 - 1 and y0 + 8 of wavefronts 0 and 1, planes z0 - 1 to z0 + zc) wraps into
    the grid, the lanes a target's x neighbours come from exist, and every node is
    stored exactly once."""
    TY, W = 8, 62
    ntx, nty, ntz = -(-nx // W), -(-ny // TY), -(-nz // zc)
    ntiles = ntx * nty * ntz
    per = -(-ntiles // 8)
    count = np.zeros((nz, ny, nx), np.int32)
    taken = np.zeros(ntiles, np.int32)
    lane = np.arange(64)
    for b in range(-(-ntiles // 8) * 8):
        tile = (b & 7) * per + (b >> 3)
        if tile >= ntiles:
            continue
        taken[tile] += 1
        tz, trow = divmod(tile, ntx * nty)
        tyi, txi = divmod(trow, ntx)
        x0, y0, z0 = txi * W, tyi * TY, tz * zc
        x = x0 - 1 + lane
        xl = wrap_axis(x, nx, True)
        assert ((xl >= 0) & (xl < nx)).all()
        for yy in (y0 - 1, y0 + TY, *range(y0, y0 + TY)):
            assert 0 <= wrap_axis(yy, ny, True) < ny
        zs = wrap_axis(np.arange(z0 - 1, z0 + zc + 1), nz, True)
        assert ((zs >= 0) & (zs < nz)).all()
        tgt = (lane >= 1) & (lane <= W) & (x < nx)
        assert ((lane[tgt] - 1 >= 0) & (lane[tgt] + 1 <= 63)).all()
        z1 = min(z0 + zc, nz)
        for w in range(TY):
            y = y0 + w
            if y < ny:
                count[z0:z1, y, x[tgt]] += 1
    assert (taken == 1).all()
    assert (count == 1).all()
