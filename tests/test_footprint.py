"""The paper's footprint and occupancy tables, reproduced by the oracle's
arithmetic and independently by the library's generic occupancy model."""
import ctypes as C
import json
import os

import pytest

from oracle import footprint as F
from paper_1711_10413_amd import dsr as D

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def test_oracle_reproduces_tables_2_and_3():
    for n, stack, pre, priv, total in GOLD["table2_scalars"]["rows"]:
        assert (F.shared_stack_scalars(n), F.PREALLOC, F.PRIVATE) == (stack, pre, priv)
        assert F.team_footprint(stack) == total
    for n, stack, pre, priv, total in GOLD["table3_arrays"]["rows"]:
        assert F.shared_stack_arrays(n) == stack and F.team_footprint(stack) == total


@pytest.mark.parametrize("table,hw", [("table4_k40_scalars", "K40"), ("table5_p100_scalars", "P100")])
def test_oracle_reproduces_scalar_occupancy(table, hw):
    h = GOLD["hardware"][hw]
    for n, static, dyn, regs, teams, smem in GOLD[table]["rows"]:
        assert F.team_footprint(F.shared_stack_scalars(n)) == static
        assert F.dynamic_global_list(n) == dyn
        t = F.teams_by_registers(regs, cap=h["max_teams_per_sm"])
        assert t == teams and t * static == smem


@pytest.mark.parametrize("table,hw", [("table6_k40_arrays", "K40"), ("table7_p100_arrays", "P100")])
def test_oracle_reproduces_array_occupancy(table, hw):
    h = GOLD["hardware"][hw]
    for n, data, static, regs, potential, smem, actual in GOLD[table]["rows"]:
        assert 96 * 4 * n == data
        assert F.team_footprint(F.shared_stack_arrays(n)) == static
        p = F.teams_by_registers(regs, cap=h["max_teams_per_sm"])
        assert p == potential and p * static == smem
        assert F.teams_actual(p, static, h["shared_per_sm"]) == actual


def test_oracle_table8_and_discussion():
    g = GOLD["table8_k40_max_regs"]
    assert [F.max_regs_for_teams(t) for t in g["teams"]] == g["max_regs"]
    d = GOLD["discussion"]
    fp = F.team_footprint(F.shared_stack_scalars(d["k40_peak_vars"]))
    assert F.teams_by_registers(d["k40_peak_regs"]) == d["k40_peak_teams"]
    assert d["k40_peak_teams"] * fp == d["k40_peak_bytes"]
    assert round(100 * d["k40_peak_bytes"] / 16384) == d["k40_peak_fraction_pct"]
    assert 65536 // (32 * 128) == d["p100_full_occupancy_regs"]


def model(hw, regs, shared, threads=128, thread_cap=1 << 30):
    # the paper's tables count registers, the block cap and shared memory
    # only (section 6.2.2); with the hardware's 2048 threads per SM the
    # P100 array rows would hold 16 teams, not the 17 Table 7 prints
    h = GOLD["hardware"][hw]
    m = D.dsr_hw_model(compute_units=1, regs_per_cu=h["regs_per_sm"], reg_granule=1,
                       max_teams_per_cu=h["max_teams_per_sm"], max_threads_per_cu=thread_cap,
                       shared_per_cu=h["shared_per_sm"], shared_granule=1)
    return D.dsr_occupancy(m, threads, regs, shared)


def test_library_model_thread_cap_on_p100():
    o = model("P100", 30, 617, thread_cap=2048)
    assert o["teams_by_registers"] == 17 and o["teams_per_cu"] == 16 and o["limiter"] == "threads"


@pytest.mark.parametrize("table,hw", [("table4_k40_scalars", "K40"), ("table5_p100_scalars", "P100")])
def test_library_model_scalar_tables(table, hw):
    for n, static, dyn, regs, teams, smem in GOLD[table]["rows"]:
        o = model(hw, regs, static)
        assert o["teams_per_cu"] == teams and o["shared_per_cu"] == smem
        assert o["limiter"] in ("registers", "teams")


@pytest.mark.parametrize("table,hw", [("table6_k40_arrays", "K40"), ("table7_p100_arrays", "P100")])
def test_library_model_array_tables(table, hw):
    for n, data, static, regs, potential, smem, actual in GOLD[table]["rows"]:
        o = model(hw, regs, static)
        assert o["teams_by_registers"] == potential and o["teams_per_cu"] == actual
        assert o["limiter"] == ("shared" if actual < potential else "registers")


def test_library_model_gfx950():
    """The same model with gfx950's parameters: 4 SIMDs x 512 VGPRs of 64
    lanes per CU, 32 workgroups and 2048 threads per CU, 160 KiB LDS; the
    registers are per SIMD, so a SIMD holds whole waves only."""
    m = D.dsr_hw_model(compute_units=256, regs_per_cu=4 * 512 * 64, reg_granule=8,
                       max_teams_per_cu=32, max_threads_per_cu=2048, shared_per_cu=163840,
                       shared_granule=128, simds_per_cu=4, wave_size=64)
    o = D.dsr_occupancy(m, 256, 158, 864 + 4096)
    assert o["teams_by_registers"] == 3 and o["teams_per_cu"] == 3 and o["limiter"] == "registers"
    o = D.dsr_occupancy(m, 256, 158, 864 + 131072)
    assert o["teams_per_cu"] == 1 and o["limiter"] == "shared"
    # 184 registers: 2 waves per SIMD, 8 per CU, so 4 two-wave teams; one
    # pooled file would hold 131072 / (184 * 128) = 5 of them
    o = D.dsr_occupancy(m, 128, 184, 864 + 16384)
    assert o["teams_by_registers"] == 4 and o["teams_per_cu"] == 4
    m.simds_per_cu = 0
    assert D.dsr_occupancy(m, 128, 184, 864 + 16384)["teams_by_registers"] == 5
