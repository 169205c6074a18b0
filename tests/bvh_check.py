"""Structural checks of an exported hierarchy (pure numpy, no GPU)."""
import numpy as np

SENTINEL = 0x7FFFFFFF


def decode(c):
    c = int(c)
    if c < 0:
        u = c & 0xFFFFFFFF
        return "leaf", u & 0x07FFFFFF, ((u >> 27) & 15) + 1
    return "node", c, 0


def check_bvh(nodes, tris, root, n_valid, verts=None, faces=None, tight=False):
    """Returns dict(depth, n_internal, leaf_sizes) or raises AssertionError.
    Checks: tree (no node reached twice), no sentinel reached, leaf runs
    partition [0, n_valid), child boxes contain everything below them,
    leaf triangles are the mesh's faces.  tight: every child box equals the
    union of the triangle boxes below it (min/max are exact, so a correct
    refit reproduces it bit for bit)."""
    ch = nodes[:, 12:14].view(np.int32)
    box = nodes[:, :12]
    seen = np.zeros(len(nodes), bool)
    covered = np.zeros(n_valid, np.int32)
    leaf_sizes = []
    depth = 0

    def tri_box(first, cnt):
        t = tris[first:first + cnt, :, :3].reshape(-1, 3)
        return t.min(0), t.max(0)

    kind, idx, cnt = decode(root)
    if kind == "leaf":
        assert idx == 0 and cnt == n_valid
        covered[:] += 1
        return {"depth": 0, "n_internal": 0, "leaf_sizes": [cnt]}
    stack = [(idx, 1)]
    n_int = 0
    while stack:
        i, d = stack.pop()
        assert 0 <= i < len(nodes), f"node index {i} out of range"
        assert not seen[i], f"node {i} reached twice"
        seen[i] = True
        n_int += 1
        depth = max(depth, d)
        assert ch[i, 0] != SENTINEL and ch[i, 1] != SENTINEL, f"node {i} was never written"
        for k in range(2):
            lo, hi = box[i, 6 * k:6 * k + 3], box[i, 6 * k + 3:6 * k + 6]
            kind, idx, cnt = decode(ch[i, k])
            if kind == "leaf":
                assert idx + cnt <= n_valid
                covered[idx:idx + cnt] += 1
                leaf_sizes.append(cnt)
                tl, th = tri_box(idx, cnt)
                assert np.all(lo <= tl) and np.all(hi >= th), f"leaf box of node {i} child {k}"
                if tight:
                    assert np.array_equal(lo, tl) and np.array_equal(hi, th), f"leaf box of node {i} child {k}"
            else:
                assert 0 <= idx < len(nodes)
                cb = box[idx]
                sub_lo = np.minimum(cb[0:3], cb[6:9])
                sub_hi = np.maximum(cb[3:6], cb[9:12])
                assert np.all(lo <= sub_lo) and np.all(hi >= sub_hi), f"box of node {i} child {k}"
                if tight:
                    assert np.array_equal(lo, sub_lo) and np.array_equal(hi, sub_hi), f"box of node {i} child {k}"
                stack.append((idx, d + 1))
    assert np.all(covered == 1), f"{int((covered != 1).sum())} triangles not in exactly one leaf"
    if verts is not None:
        fid = tris[:, 0, 3].view(np.int32)
        assert len(np.unique(fid)) == n_valid
        for k in range(3):
            assert np.array_equal(tris[:, k, :3], verts[faces[fid, k]])
    return {"depth": depth, "n_internal": n_int, "leaf_sizes": leaf_sizes}
