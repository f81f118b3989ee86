"""Kernel-name normalisation of the rocprofv3 summaries: mangled and
demangled names of one kernel instantiation map to one key."""
from paper_2512_01027_amd.profsum import short


def test_mangled_and_demangled_names_agree():
    assert short("_ZN5pulbm9k_collideILi4EDF16_Lb0EEEvNS_7CaseTabEPKii") == "pulbm::k_collide<4, _Float16, false>"
    assert short("_ZN5pulbm9k_collideILi3EfLb1EEEvNS_7CaseTabEPKii") == "pulbm::k_collide<3, float, true>"
    assert short("_ZN5pulbm9k_momentsILi2EDF16_EEvNS_7CaseTabEPKii") == "pulbm::k_moments<2, _Float16>"
    assert short("void pulbm::k_collide<3, float, false>(pulbm::CaseTab, int const*, int)") == \
        "pulbm::k_collide<3, float, false>"
