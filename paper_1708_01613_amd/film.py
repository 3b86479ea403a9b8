"""The two-bubble film workload of Sec. 4 (Table 2, Fig. 7 and Fig. plot) in
lattice units, and the foam statistics of Sec. 5 (Table 5) over a run.

Two equal bubbles in line with a thin liquid film between them, on a periodic
D2Q9 (or D3Q19) lattice with the film barrier and the rupture test on.  The
run records, every `every` steps, what the paper plots and reports:

* the bulk pressure p0 and the velocity component along a line across the
  film, through its centre and perpendicular to the line of centres (the
  "vertical line in the middle of two bubbles" of Fig. plot), and the
  density along the line of centres (the film's thickness profile);
* a probe in the film half a radius off its centre, where the drainage flow
  runs along the film: its along-film velocity, whose sign changes before the
  rupture are the velocity oscillation the abstract names (a diagnostic, not
  a gate of the rupture test);
* the number of bubbles, the rupture events so far and the foam statistics.

All fields come from the library's queries (flb_get_density, flb_get_pressure,
flb_get_velocity, flb_get_labels, flb_get_rupture_events, flb_get_foam_stats);
this module only samples and arranges them.  `sim` may be any object with
those queries under the names the binding's `Sim` gives them.

Table 2 maps to lattice units at 4 cells per mm: a 45 mm domain is 180
cells, an 8 mm bubble a radius of 16 cells.
"""
import numpy as np

CELLS_PER_MM = 4


def table2_geometry(gap=3.0, cells_per_mm=CELLS_PER_MM, lattice=0):
    """Lattice size and nuclei of Table 2's two in-line bubbles (8 mm in a
    45 mm domain) with `gap` cells of liquid between them."""
    n = int(round(45 * cells_per_mm))
    r = 8 * cells_per_mm / 2.0
    c = n / 2.0
    x1, x2 = c - r - gap / 2.0 - 0.5, c + r + gap / 2.0 + 0.5
    z = c if lattice == 1 else 0.0
    return n, [[x1, c, z, r], [x2, c, z, r]]


def _line_x(field, x, y, z):
    """Values along y at fixed x (and z) of a (ny, nx) or (nz, ny, nx) field."""
    return field[:, x] if field.ndim == 2 else field[z, :, x]


def _row(field, y, z):
    return field[y] if field.ndim == 2 else field[z, y]


def sample(sim, centres, radius):
    """One record of the film between bubbles centred at centres[0] and
    centres[1] (lattice coordinates, the line of centres along x)."""
    (x1, y1, z1), (x2, _, _) = centres
    xm, ym, zm = int(round((x1 + x2) / 2.0)), int(round(y1)), int(round(z1))
    rho = sim.density()
    p = sim.pressure()
    u = sim.velocity()
    uy = u[1]
    _, nb = sim.labels()
    events = sim.rupture_events()
    probe_y = ym + int(round(radius / 2.0))
    return {
        "n_bubbles": int(nb),
        # distinct (step, pair) records: a log may repeat one pair within a step
        "events": len({tuple(int(v) for v in e) for e in events}),
        "first_event_step": int(min(e[0] for e in events)) if len(events) else None,
        "centre_density": float(rho[ym, xm] if rho.ndim == 2 else rho[zm, ym, xm]),
        "centre_pressure": float(p[ym, xm] if p.ndim == 2 else p[zm, ym, xm]),
        "probe_velocity": float(uy[probe_y, xm] if uy.ndim == 2 else uy[zm, probe_y, xm]),
        "line_pressure": _line_x(p, xm, ym, zm).copy(),
        "line_velocity": _line_x(uy, xm, ym, zm).copy(),
        "centres_density": _row(rho, ym, zm).copy(),
        "foam": sim.foam_stats(),
    }


def sign_changes(values):
    """Sign changes along a sequence, zeros skipped."""
    s = np.sign(np.asarray(values, np.float64))
    s = s[s != 0]
    return int(np.count_nonzero(s[1:] != s[:-1]))


def run(sim, nuclei, steps, every):
    """Advances `sim` (already holding the nuclei's initial state) by
    `steps` steps and records a sample every `every` steps (and at step 0).
    Returns the records and a summary: the first rupture step, the first
    sampled step with one bubble, the velocity sign changes at the probe
    before the rupture, and the profiles of the last sample before and the
    first sample after the rupture."""
    centres = [tuple(n[:3]) for n in nuclei[:2]]
    radius = float(nuclei[0][3])
    recs = [dict(step=0, **sample(sim, centres, radius))]
    done = 0
    while done < steps:
        k = min(every, steps - done)
        sim.step(k)
        done += k
        recs.append(dict(step=done, **sample(sim, centres, radius)))
    rupture = next((r["first_event_step"] for r in recs if r["first_event_step"] is not None), None)
    merged = next((r["step"] for r in recs if r["n_bubbles"] == 1), None)
    before = [r for r in recs if rupture is None or r["step"] <= rupture]
    after = [r for r in recs if rupture is not None and r["step"] > rupture]
    summary = {
        "rupture_step": rupture,
        "merged_by_step": merged,
        "probe_sign_changes_before_rupture": sign_changes([r["probe_velocity"] for r in before]),
        "profile_before": {k: before[-1][k] for k in ("line_pressure", "line_velocity")} if before else None,
        "profile_after": {k: after[0][k] for k in ("line_pressure", "line_velocity")} if after else None,
        "foam_first": recs[0]["foam"],
        "foam_last": recs[-1]["foam"],
    }
    return recs, summary
