"""The paper-table rows are set up as the paper states them (Sec. 4):
Shakhov (ES-BGK for Table 4), M = 5 (10 in Table 3 and the M = 10 rows of
Table 4), Tol 1e-8, CFL 0.9, s1 = s2 = 2, s3 = 4, coarsest grid 8x8,
lid speed 50 m/s at 273 K, and the per-section walls (host logic only)."""
import math

from paper_2206_13164_amd import paper_tables as T


def test_rows_follow_the_papers_setup():
    for table, label, kw, paper in T.ROWS:
        s = T.row_spec(kw)
        model = 2 if table == "4" else 1  # Table 4: ES-BGK, beta = Pr (Sec. 4)
        M = 10 if "M = 10" in label else 5
        assert (table != "3") or M == 10, label  # Table 3 lists M >= 10 only
        assert (s["M"], s["collision"], s["tol"], s["cfl"]) == (M, model, 1e-8, 0.9), label
        assert s["beta"] == (2.0 / 3.0 if model == 2 else 1.0), label
        assert (s["s1"], s["s2"], s["s3"], s["gamma"]) == (2, 2, 4, 1), label
        assert s["nx"] == s["ny"] and s["nx"] >> (s["levels"] - 1) == 8, label
        assert abs(s["Pr"] - 2.0 / 3.0) < 1e-15
        assert s["order"] == (2 if table == "9" else 1), label
        assert (paper[0] is None) == (table == "9"), label  # Euler diverges at 2nd order
        uS, uE, uN, uW = s["wall_u"]
        if table == "6":   # anti-parallel four-sided motion
            assert uN == -uS == uE == -uW == T.U_W
        elif table == "8":  # bottom heated to twice the other walls' temperature, static
            assert s["wall_u"] == [0.0] * 4 and s["wall_theta"] == [2.0, 1.0, 1.0, 1.0]
        else:               # single lid moving right
            assert s["wall_u"] == [0.0, 0.0, T.U_W, 0.0] and s["wall_theta"] == [1.0] * 4


def test_lid_speed_is_50_m_per_s_at_273_K_in_argon_units():
    # U_W / sqrt(R T0) with R = k_B / m_Ar (the constant keeps four digits)
    R = 1.380649e-23 / (39.948 * 1.66053906660e-27)
    assert abs(50.0 / math.sqrt(R * 273.0) - T.U_W) < 1e-4
