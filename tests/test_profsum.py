"""Kernel-name normalisation of the rocprofv3 summaries: mangled and
demangled names of one kernel instantiation map to one key."""
from paper_2512_01027_amd.profsum import short


def test_mangled_and_demangled_names_agree():
    assert short("_ZN5pulbm9k_collideILi4EDF16_Lb0EEEvNS_7CaseTabEPKii") == "pulbm::k_collide<4, _Float16, false>"
    assert short("_ZN5pulbm9k_collideILi3EfLb1EEEvNS_7CaseTabEPKii") == "pulbm::k_collide<3, float, true>"
    assert short("_ZN5pulbm9k_momentsILi2EDF16_EEvNS_7CaseTabEPKii") == "pulbm::k_moments<2, _Float16>"
    assert short("void pulbm::k_collide<3, float, false>(pulbm::CaseTab, int const*, int)") == \
        "pulbm::k_collide<3, float, false>"
    # the collide kernels of each step parity
    assert short("_ZN5pulbm9k_collideILi3EDF16_Lb0ELi1EEEvPKPNS_7CaseDevEPKii") == \
        "pulbm::k_collide<3, _Float16, false, 1>"
    assert short("pulbm::k_collide<3, float, false, 0>(pulbm::CaseDev* const*, int const*, int)") == \
        "pulbm::k_collide<3, float, false, 0>"


def test_issue_summary_per_wave_and_issue_time(tmp_path):
    """Two dispatches of one kernel: counters are averaged over dispatches,
    divided by SQ_WAVES, and the VALU issue time is
    waves x VALU/wave x 4 cycles / (1024 SIMDs x 2.4 GHz)."""
    from paper_2512_01027_amd.profsum import issue
    sq, tr = tmp_path / "sq", tmp_path / "tr"
    sq.mkdir()
    tr.mkdir()
    name = "void pulbm::k_pressure<3, float>(pulbm::CaseTab, int const*, int)"
    rows = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
    for d in (1, 2):
        rows += [f'{d},"{name}",SQ_WAVES,32768', f'{d},"{name}",SQ_INSTS_VALU,{32768 * (300 + 2 * (d - 1))}',
                 f'{d},"{name}",SQ_INSTS_LDS,{32768 * 60}', f'{d},"{name}",SQ_INSTS_SALU,{32768 * 170}']
    (sq / "run_counter_collection.csv").write_text("\n".join(rows) + "\n")
    (tr / "run_kernel_stats.csv").write_text(
        "Name,Calls,TotalDurationNs,AverageNs,Percentage,MinNs,MaxNs\n"
        f'"{name}",2,48000,24000,100.0,23000,25000\n')
    lines = issue(str(sq), str(tr)).splitlines()
    assert len(lines) == 2
    cells = [c.strip() for c in lines[1].split("|")]
    assert cells[0] == "pulbm::k_pressure<3, float>"
    assert cells[1:5] == ["32768", "301", "60", "170"]
    t_issue = 32768 * 301 * 4 / (1024 * 2.4e9) * 1e6
    assert abs(float(cells[5]) - t_issue) < 0.05
    assert cells[6] == "24.00"
    assert abs(float(cells[7]) - t_issue / 24.0) < 0.005
