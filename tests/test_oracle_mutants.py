"""Each pin must be able to fail: plant one plausible mistake at a time in a
copy of the oracle source (a flipped sign, a dropped term, a wrong index, a
transposed operand), rebuild the copy, and check that the pin battery
rejects it.  The oracle itself is never modified."""
import os

import pytest

import oracle
import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "rti_oracle.c")

MUTANTS = {
    "mass: divergence sign": (
        "- r * ((L->M[XF(L, i + 1, j)] - L->M[XF(L, i, j)])",
        "+ r * ((L->M[XF(L, i + 1, j)] - L->M[XF(L, i, j)])"),
    "mass: dropped N term": (
        "+ (L->N[YF(L, i, j + 1)] - L->N[YF(L, i, j)]));",
        "+ 0.0 * (L->N[YF(L, i, j + 1)] - L->N[YF(L, i, j)]));"),
    "mass: no clip to the ground": ("if (hh + e < 0.0) {", "if (0) {"),
    "pressure: sign": (
        "(gr * D) * (L->eta[CELL(L, i, j)] - L->eta[CELL(L, i - 1, j)])",
        "(gr * D) * (L->eta[CELL(L, i - 1, j)] - L->eta[CELL(L, i, j)])"),
    "pressure: dropped depth": (
        "const double P = (gr * D) * (L->eta[CELL(L, i, j)] - L->eta[CELL(L, i - 1, j)]);",
        "const double P = (gr) * (L->eta[CELL(L, i, j)] - L->eta[CELL(L, i - 1, j)]);"),
    "pressure: y uses the x neighbour": (
        "(gr * D) * (L->eta[CELL(L, i, j)] - L->eta[CELL(L, i, j - 1)])",
        "(gr * D) * (L->eta[CELL(L, i, j)] - L->eta[CELL(L, i - 1, j)])"),
    "advection: downwind": (
        "if (s > 0.0) return okm ? v - vm : 0.0;\n    if (s < 0.0) return okp ? vp - v : 0.0;",
        "if (s > 0.0) return okp ? vp - v : 0.0;\n    if (s < 0.0) return okm ? v - vm : 0.0;"),
    "advection: dropped cross term": ("const double A = r * (X + Y);", "const double A = r * X;"),
    "advection: cross flux uses M twice": (
        "const double Y = upwind_diff(nb, (m * nb) * rD,", "const double Y = upwind_diff(nb, (m * m) * rD,"),
    "advection: neighbour quotient by the face's own depth": (
        "okm ? (mm * mm) * (1.0 / Dm) : 0.0", "okm ? (mm * mm) * rD : 0.0"),
    "advection: N average index": (
        "return 0.25 * ((L->N[YF(L, i - 1, j)] + L->N[YF(L, i - 1, j + 1)])",
        "return 0.25 * ((L->N[YF(L, i - 1, j)] + L->N[YF(L, i - 1, j)])"),
    "friction: factor 1 instead of 1/2": (
        "const double fc = 0.5 * d->dt * d->g * d->manning * d->manning;",
        "const double fc = d->dt * d->g * d->manning * d->manning;"),
    "friction: D^(4/3)": ("return s * ((rD * rD) * ora_cbrt_rn(rD));", "return s * (rD * ora_cbrt_rn(rD));"),
    "cube root: libm's value kept": ("    double y = cbrt(x);\n    for (int moves", "    double y = cbrt(x);\n    return y;\n    for (int moves"),
    "cube root: midpoint exponent": ("const int sh = ex - (3 * e - 3);", "const int sh = ex - (3 * e - 2);"),
    "source: rotation sign": (
        "double xp = ddx * ct + ddy * st;\n                double yp = -(ddx * st) + ddy * ct;",
        "double xp = ddx * ct - ddy * st;\n                double yp = ddx * st + ddy * ct;"),
    "source: a and b as full axes": ("double u = xp / a, v = yp / b;", "double u = xp / (0.5 * a), v = yp / (0.5 * b);"),
    "source: Gaussian scale": ("s = amp * exp(-0.5 * rho2);", "s = amp * exp(-rho2);"),
    "source: land cells get the displacement": ("double e = (h > 0.0) ? s : -h;", "double e = s;"),
    "child->parent: transposed parent cell": (
        "size_t pc = CELL(P, C->off_i + I, C->off_j + J);", "size_t pc = CELL(P, C->off_j + J, C->off_i + I);"),
    "child->parent: dry cells in the mean": (
        "if (C->h[CELL(C, ii, jj)] + e > d->eps) { s += e; k++; }", "{ s += e; k++; }"),
    "child->parent: two columns summed": (
        "for (int ii = 3 * I; ii < 3 * I + 3; ii++)", "for (int ii = 3 * I; ii < 3 * I + 2; ii++)"),
    "parent->child: x-face of the cell to the west": (
        "C->M[XF(C, 3 * I, 3 * J + k)] = P->M[XF(P, I0 + I, J0 + J)];",
        "C->M[XF(C, 3 * I, 3 * J + k)] = P->M[XF(P, I0 + I - 1, J0 + J)];"),
    "parent->child: y-face one row up": (
        "C->N[YF(C, 3 * I + k, 3 * J)] = P->N[YF(P, I0 + I, J0 + J)];",
        "C->N[YF(C, 3 * I + k, 3 * J)] = P->N[YF(P, I0 + I, J0 + J + 1)];"),
    "parent->child: faces inside the footprint injected too": (
        "if (covered(C, I - 1, J) != covered(C, I, J))", "if (covered(C, I - 1, J) || covered(C, I, J))"),
    "parent->child: child rows of a face": (
        "C->M[XF(C, 3 * I, 3 * J + k)]", "C->M[XF(C, 3 * I, 3 * J + k / 2)]"),
    "mask: faces to outside cells active": (
        "    if (!inside(L, i - 1, j) || !inside(L, i, j)) return 0;\n", ""),
    "mask: outside cells updated": ("            if (!inside(L, i, j)) continue;\n            double e", "            double e"),
    "child->parent: ring of the rectangle, not of the covered region": (
        "if (!covered(C, I + di, J + dj)) ring = 1;",
        "if (I + di < 0 || J + dj < 0 || I + di >= fw || J + dj >= fh) ring = 1;"),
    "open boundary: west sign": (
        "radiate(d, L->h[CELL(L, 0, j)], L->eta[CELL(L, 0, j)], -1.0);",
        "radiate(d, L->h[CELL(L, 0, j)], L->eta[CELL(L, 0, j)], 1.0);"),
    "maxima: level instead of depth on land": ("double v = (h > 0.0) ? e : h + e;", "double v = e;"),
}

BATTERY = [pins.pin_cbrt_rn, pins.pin_source, pins.pin_lake_at_rest, pins.pin_closed_mass, pins.pin_nested_mass, pins.pin_jnz_linear,
           pins.pin_max_tracking, pins.pin_open_boundary, pins.pin_dispersion, pins.pin_mirror_symmetry,
           pins.pin_friction_ode, pins.pin_dam_break, pins.pin_consistency, pins.pin_masked_subrect,
           pins.pin_masked_blocks, pins.pin_masked_mass, pins.pin_nest_locality]


def test_unmodified_copy_passes(tmp_path):
    src = open(SRC).read()
    path = tmp_path / "copy.c"
    path.write_text(src)
    lib = oracle.load_variant(str(path), str(tmp_path / "copy.so"))
    for pin in BATTERY:
        pin(lib=lib, quick=True)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    find, repl = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(find) >= 1, f"mutation site not found: {find}"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(find, repl))
    lib = oracle.load_variant(str(path), str(tmp_path / "mutant.so"))
    caught = None
    for pin in BATTERY:
        try:
            pin(lib=lib, quick=True)
        except (AssertionError, FloatingPointError, ValueError) as e:
            caught = f"{pin.__name__}: {e}"
            break
    assert caught is not None, f"no pin caught the planted mistake '{name}'"
    print(f"[{name}] caught by {caught}")
