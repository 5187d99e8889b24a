"""Each planted mistake in a copy of the oracle must make some pin fail.

The mutations are the plausible slips of a hand translation of the paper's
formulas: a dropped or flipped term, a wrong sign or index, a transposed
operand, a changed boundary convention.  Every mutant is compiled from a
patched copy of ``oracle/oracle.c`` in a temporary directory; the real
oracle is never touched.
"""
import os

import pytest

import oracle as oracle_mod
import oracle_pins

SRC = os.path.join(os.path.dirname(oracle_mod.__file__), "oracle.c")

# (name, original text, mutated text, which occurrence: 0 = first)
MUTANTS = [
    ("centroid_sign", "Sx = Sx + (vx + wx) * Ai;", "Sx = Sx + (vx - wx) * Ai;"),
    ("centroid_six", "g0[0] = Sx / (6.0 * a);", "g0[0] = Sx / (3.0 * a);"),
    ("centroid_half_area", "double a = 0.5 * S;", "double a = S;"),
    ("partial_area_transposed", "double Ai = wx * vy - vx * wy;", "double Ai = vx * vy - wx * wy;"),
    ("gen_b_sign", "double b = wx - vx;", "double b = vx - wx;"),
    ("gen_c_dropped_term", "double c = -(a * vx + b * vy);", "double c = -(a * vx);"),
    ("gen_w12_sign", "double w12 = (-2.0 * a) * b;", "double w12 = (2.0 * a) * b;"),
    ("gen_e_index", "double ey = (-2.0 * c) * b;", "double ey = (-2.0 * c) * a;"),
    ("gen_d_transposed", "double dy = w12 * g0[0] + w22 * g0[1];",
     "double dy = w12 * g0[1] + w22 * g0[0];"),
    ("gen_den_sign", "double den = a * a + b * b;", "double den = a * a - b * b;"),
    ("sqdist_index", "return dx * dx + dy * dy;", "return dx * dx + dx * dy;"),
    ("voronoi_strict", "if (!(M0 <= Mi)) in = 0;", "if (!(M0 < Mi)) in = 0;"),
    ("soo_nonstrict", "if (LHS < RHS) count += 1;", "if (LHS <= RHS) count += 1;"),
    ("soo_rhs_sign", "double RHS = V[2 * j + 1] * dVx - V[2 * j] * dVy;\n            if (LHS < RHS)",
     "double RHS = V[2 * j + 1] * dVx + V[2 * j] * dVy;\n            if (LHS < RHS)"),
    ("ray_printed_parity", "(crossings % 2) == 1", "(crossings % 2) == 0"),
    ("ray_going_up", "int going_up = V[2 * i + 1] > V[2 * j + 1];",
     "int going_up = V[2 * i + 1] < V[2 * j + 1];"),
    ("ray_in_range_closed", "int in_range = (V[2 * i + 1] > py) != (V[2 * j + 1] > py);",
     "int in_range = (V[2 * i + 1] >= py) != (V[2 * j + 1] > py);"),
    ("pose_rotation_sign", "W[2 * i] = (c * vx - s * vy) + tx;", "W[2 * i] = (c * vx + s * vy) + tx;"),
    ("raster_transposed", "isin[j * width + i] = (uint8_t)in;", "isin[i * height + j] = (uint8_t)in;"),
    ("raster_row_offset", "double py = y0 + (double)j * dy;", "double py = y0 + (double)(j + 1) * dy;"),
    ("raster_x_step", "double px = x0 + (double)i * dx;", "double px = x0 + (double)i * dy;"),
    ("locate_last_wins", "for (int64_t k = 0; k < P && id < 0; ++k) {", "for (int64_t k = 0; k < P; ++k) {"),
    ("locate_generator_offset", "const double *Pk = G + 2 * (vtx_off[k] + k);",
     "const double *Pk = G + 2 * vtx_off[k];"),
    ("allpairs_bit_order", "row[j >> 5] |= (uint32_t)1u << (j & 31);",
     "row[j >> 5] |= (uint32_t)1u << (31 - (j & 31));"),
    ("cost_body_frame_sign", "double by = (-s) * dx + c * dy;\n        double best = 0.0;",
     "double by = s * dx + c * dy;\n        double best = 0.0;"),
    ("normalized_margin_scale", "return -(M0 - Mi) / (2.0 * len);", "return -(M0 - Mi) / len;"),
    ("grad_theta_swap", "double cth = gpx * by + gpy * (-bx);",
     "double cth = gpx * bx + gpy * (-by);"),
    ("grad_t_sign", "double ctx_ = -(c * gpx - s * gpy);", "double ctx_ = -(c * gpx + s * gpy);"),
    ("grad_b_sign", "double cbx = sigma * (ry / L - f * ex / L3);",
     "double cbx = sigma * (ry / L + f * ex / L3);"),
    ("grad_a_index", "double cay = sigma * ((rx - ex) / L + f * ey / L3);",
     "double cay = sigma * ((rx - ey) / L + f * ey / L3);"),
    ("cost_argmin_tie_last", "\n            if (i == 0 || d < best) {",
     "\n            if (i == 0 || d <= best) {"),
    ("grad_argmin_tie_last", "\n                if (i == 0 || d < best) {",
     "\n                if (i == 0 || d <= best) {"),
    ("pieces_first_decides", "                if (all) in = 1;", "                in = all;\n                break;"),
    ("pieces_skip_last", "for (int64_t k = 0; k < K && !in; ++k) {",
     "for (int64_t k = 0; k + 1 < K && !in; ++k) {"),
    ("pieces_generator_offset", "const double *Pk = G + 2 * (off[k] + k);",
     "const double *Pk = G + 2 * off[k];"),
    ("pieces_gather_index", "W[2 * j] = V[2 * idx[off[k] + j]];", "W[2 * j] = V[2 * (off[k] + j)];"),
    ("pieces_open", "if (!(M0 <= Mi)) all = 0;", "if (!(M0 < Mi)) all = 0;"),
    ("cost_state_off_by_one", "if (state) state[j] = (int32_t)arg;",
     "if (state) state[j] = (int32_t)arg + 1;"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mutated = src.replace(old, new, 1)
    p = tmp_path / "oracle_mut.c"
    p.write_text(mutated)
    lib = oracle_mod.build(str(p), str(tmp_path / f"lib_{name}.so"))
    o = oracle_mod.Oracle(lib)
    failed = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(o)
        except AssertionError:
            failed.append(pin.__name__)
            break
        except Exception as e:  # a crash on a nonsense value also counts
            failed.append(f"{pin.__name__}:{type(e).__name__}")
            break
    assert failed, f"no pin caught mutant {name}"
