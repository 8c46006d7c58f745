"""The strip kernel's work decomposition, modelled on the CPU.

A Python restatement of the index arithmetic of k_step_strip / strip_body
(strip order, the 62 output chunks of a wavefront, wrapped or wall source
chunks and rows, clamped loads, stores redirected to the trash area) checks,
for many shapes and every launch configuration, that every load and store
stays inside the grid's allocation and that every node is written exactly
once.  It needs no GPU; it guards the decomposition, not the arithmetic.
"""
import pytest


def layout(nx, ny, c, snapshot=True):
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
    off += 3 * 1024
    return dict(pitch=pitch, rs=rs, field_off=field_off, state=state, flags_off=flags_off,
                trash_off=trash_off, total=off)


def wrap_axis(c, n, periodic):
    if 0 <= c < n:
        return c
    if not periodic:
        return -1
    return c % n


def run_model(nx, ny, c, VEC, NY, waves, periodic, cus=256):
    L = layout(nx, ny, c)
    px, py = periodic & 1, periodic & 2
    nch = nx // VEC
    strips_x = (nch + 61) // 62
    strips_y = (ny + NY - 1) // NY
    units = (strips_x * strips_y + 3) // 4
    if waves > 0:
        blocks = min(max(8, (cus * waves // 4) // 8 * 8), (units + 7) // 8 * 8)
    else:
        blocks = (units + 7) // 8 * 8
    per_xcd = (units + 7) // 8
    written = {}
    p = 0
    src = [p * L["state"] + L["field_off"][q] for q in range(3)]
    dst = [(1 - p) * L["state"] + L["field_off"][q] for q in range(3)]
    for b in range(blocks):
        xcd, local = b & 7, b >> 3
        begin, end = xcd * per_xcd, min(units, xcd * per_xcd + per_xcd)
        stride = blocks >> 3 if waves > 0 else units
        u = begin + local
        while u < end:
            for wave in range(4):
                s = u * 4 + wave
                sy, sx = divmod(s, strips_x)
                if sy >= strips_y:
                    continue
                chunk0, y0 = sx * 62, sy * NY
                for lane in range(64):
                    ch = chunk0 - 1 + lane
                    col_ok = 0 <= ch < nch or bool(px)
                    xc = (ch % nch) * VEC if col_ok else 0
                    lane_out = 1 <= lane <= 62 and ch < nch
                    for i in range(NY + 2):
                        rr = wrap_axis(y0 - 1 + i, ny, py)
                        row = rr if rr >= 0 else 0
                        assert 0 <= row < ny
                        for q in range(3):
                            lo = src[q] + (row * L["rs"] + xc) * c
                            assert 0 <= lo and lo + VEC * c <= src[q] - L["field_off"][q] + L["state"]
                        assert xc + VEC <= L["pitch"]
                        if i >= 2:
                            t = y0 + i - 2
                            ok = t < ny and lane_out
                            for q in range(3):
                                if ok:
                                    lo = dst[q] + (t * L["rs"] + ch * VEC) * c
                                    key = (q, t, ch)
                                    written[key] = written.get(key, 0) + 1
                                else:
                                    lo = L["trash_off"] + q * 1024 + lane * VEC * c
                                    assert lo + VEC * c <= L["trash_off"] + 3 * 1024
                                assert 0 <= lo and lo + VEC * c <= L["total"]
            u += stride
    return written, nch


SHAPES = [(512, 77, 0), (512, 77, 3), (264, 61, 0), (264, 61, 1), (264, 61, 2), (17, 9, 3),
          (3, 3, 3), (3, 3, 0), (64, 32, 1), (124, 30, 3), (130, 5, 2)]


@pytest.mark.parametrize("nx,ny,periodic", SHAPES)
def test_every_node_written_once_and_all_accesses_in_bounds(nx, ny, periodic):
    for c, vecs in ((8, (1, 2)), (4, (1, 2, 4)), (2, (1, 2, 4, 8))):
        for VEC in vecs:
            if nx % VEC:
                continue
            for NY in (6, 14):
                for waves in (0, 8):
                    written, nch = run_model(nx, ny, c, VEC, NY, waves, periodic)
                    assert len(written) == 3 * ny * nch, (nx, ny, VEC, NY, waves)
                    assert set(written.values()) == {1}
