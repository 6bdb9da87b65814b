"""Pin of the oracle's ghost-value rule (Sec. 2.2 and its figure of the
affected points): a ghost node is extrapolated along every coordinate line
on which it has a fluid neighbour and enough consecutive fluid nodes behind
that neighbour (four for the fourth-order stencil, three for the
third-order ones), and takes the unweighted mean of those one-dimensional
extrapolations; a ghost with no such line is a geometry error.

A hand-built nonconvex solid (a block with a two-node-wide notch) on a
16 x 16 grid, with a control point on every fluid-ghost edge at a chosen
distance, covers the figure's cases: (a) one fluid neighbour, one line;
(b) two fluid neighbours at a corner, the mean of two lines; (c, d) two
fluid neighbours but the line across the notch too short, the other line
only.  The valid lines of each ghost are listed by hand below.  The field
is not a polynomial, so the lines disagree and the unweighted mean is told
apart from any other weighting; each line's value is the polynomial through
its points (numpy.polyfit), evaluated at the ghost."""
import numpy as np
import pytest

from oracle import geometry as OG

NX = NY = 16
H = 0.1


def _field(x, y):
    return np.exp(0.7 * x) * np.cos(1.3 * y) + np.sin(2.1 * x * y)


def _mask(notch_depth):
    """Fluid mask: solid block i, j in [4, 11] with a notch at i in {7, 8}
    from the top row down `notch_depth` rows (four fluid nodes lie between
    the block and every grid edge)."""
    solid = np.zeros((NY, NX), dtype=bool)
    solid[4:12, 4:12] = True
    solid[12 - notch_depth:12, 7:9] = False
    # one solid node at the grid edge, three fluid nodes left of the block's
    # corner row: that line suits the three-point stencils only
    solid[4, 0] = True
    return ~solid


def _hand_geometry(fluid):
    """An oracle Geometry holding only what the ghost operator reads: node
    classes from the mask and one control point per fluid-ghost edge."""
    g = OG.Geometry.__new__(OG.Geometry)
    g.nx, g.ny, g.h = NX, NY, H
    g.fluid = fluid
    solid = ~fluid
    pad = np.zeros((NY + 2, NX + 2), dtype=bool)
    pad[1:-1, 1:-1] = fluid
    ghost = solid & (pad[1:-1, 2:] | pad[1:-1, :-2] | pad[2:, 1:-1] | pad[:-2, 1:-1])
    gj, gi = np.nonzero(ghost)
    g.ng, g.g_i, g.g_j = gi.size, gi, gj
    gid = {(i, j): k for k, (i, j) in enumerate(zip(gi, gj))}
    ax, sg, cif, cjf, th = [], [], [], [], []
    g.g_ctrl = [[] for _ in range(g.ng)]
    rng = np.random.default_rng(7)
    for k, (i, j) in enumerate(zip(gi, gj)):
        for axis, di, dj in ((0, 1, 0), (0, -1, 0), (1, 0, 1), (1, 0, -1)):
            fi, fj = i + di, j + dj
            if 0 <= fi < NX and 0 <= fj < NY and fluid[fj, fi]:
                g.g_ctrl[k].append(len(ax))
                ax.append(axis)
                sg.append(-(di + dj))       # ghost = fluid + sigma along the axis
                cif.append(fi)
                cjf.append(fj)
                th.append(rng.uniform(0.2, 0.95))
    g.nc = len(ax)
    g.c_axis, g.c_sigma = np.array(ax), np.array(sg)
    g.c_if, g.c_jf, g.c_theta = np.array(cif), np.array(cjf), np.array(th)
    return g, gid


def _control_xy(g, c):
    x, y = g.c_if[c] * H, g.c_jf[c] * H
    d = g.c_sigma[c] * g.c_theta[c] * H
    return (x + d, y) if g.c_axis[c] == 0 else (x, y + d)


def _line_value(g, c, kind):
    """Value at the ghost (+1) of the polynomial through the line's points:
    control point at theta and fluid nodes at -1, -2, ... (with the wall
    value), or fluid nodes at 0, -1, -2 (without)."""
    s = g.c_sigma[c]
    node = lambda m: ((g.c_if[c] - m * s) * H, g.c_jf[c] * H) if g.c_axis[c] == 0 else \
        (g.c_if[c] * H, (g.c_jf[c] - m * s) * H)
    if kind == OG.KIND_3N:
        t = [0.0, -1.0, -2.0]
        v = [_field(*node(m)) for m in (0, 1, 2)]
    else:
        count = 4 if kind == OG.KIND_4B else 3
        t = [g.c_theta[c]] + [-float(m) for m in range(1, count)]
        v = [_field(*_control_xy(g, c))] + [_field(*node(m)) for m in range(1, count)]
    return np.polyval(np.polyfit(t, v, len(t) - 1), 1.0)


# Valid lines, by hand, for the notch of depth 1 (fluid nodes (7, 11) and
# (8, 11) cut into the block's top row).  Keys: ghost (i, j) -> fluid
# neighbours whose lines are valid, for the three-point and the four-point
# stencils.
CASES = {
    # (a) the notch floor: one fluid neighbour above, open fluid behind it
    (7, 10): ([(7, 11)], [(7, 11)]),
    (8, 10): ([(8, 11)], [(8, 11)]),
    # (c, d) the notch walls: fluid across the notch is only two nodes wide,
    # so the horizontal line is never valid, the vertical one is
    (6, 11): ([(6, 12)], [(6, 12)]),
    (9, 11): ([(9, 12)], [(9, 12)]),
    # (b) corners of the block: both lines open
    (4, 4): ([(3, 4), (4, 3)], [(4, 3)]),     # three fluid nodes to the left
    (0, 4): ([(1, 4), (0, 3), (0, 5)], [(0, 3), (0, 5)]),   # the lone node: three lines
    (11, 11): ([(12, 11), (11, 12)], [(12, 11), (11, 12)]),
    (11, 4): ([(12, 4), (11, 3)], [(12, 4), (11, 3)]),
    # plain sides: one line
    (4, 7): ([(3, 7)], [(3, 7)]),
    (9, 4): ([(9, 3)], [(9, 3)]),
}


@pytest.mark.parametrize("kind", [OG.KIND_3B, OG.KIND_3N, OG.KIND_4B])
def test_valid_lines_and_unweighted_mean(kind):
    g, gid = _hand_geometry(_mask(1))
    Ef, Eb, nvalid = g._ghost_operator(kind)
    f_nodes = np.array([[_field(i * H, j * H) for i in range(NX)] for j in range(NY)]).ravel()
    f_ctrl = np.array([_field(*_control_xy(g, c)) for c in range(g.nc)])
    got = Ef @ f_nodes + (Eb @ f_ctrl if kind != OG.KIND_3N else 0.0)
    checked = 0
    for (i, j), (lines3, lines4) in CASES.items():
        k = gid[(i, j)]
        lines = lines4 if kind == OG.KIND_4B else lines3
        valid = [c for c in g.g_ctrl[k] if (g.c_if[c], g.c_jf[c]) in lines]
        assert nvalid[k] == len(lines) == len(valid), ((i, j), nvalid[k], lines)
        vals = [_line_value(g, c, kind) for c in valid]
        assert got[k] == pytest.approx(np.mean(vals), abs=1e-12), (i, j)
        if len(vals) >= 2:
            # the lines disagree by far more than rounding: the weighting matters
            assert np.ptp(vals) > 1e-5, (i, j, vals)
        checked += 1
    assert checked == len(CASES)


def test_ghost_without_a_valid_line_is_an_error():
    """A notch two rows deep: the ghosts on its walls below the top row have
    a fluid neighbour only across the two-node notch, no valid line."""
    g, gid = _hand_geometry(_mask(2))
    with pytest.raises(OG.GeometryError, match="no valid"):
        g._ghost_operator(OG.KIND_3B)
