"""Kernel names in rocprofv3 summaries: every kernel of the hot path maps to
the name the library's own profiler gives it (CPU only)."""
from paper_2507_01958_amd.profiling import classify

NS = "void mfg::(anonymous namespace)::"


def _c(*names):
    return classify([NS + n for n in names])


def test_stencil_and_pcg_kernels():
    assert _c("k_AAt_tile<true, true, 1>(mfg::AatArgs)",
              "k_AAt_tile<true, false, 2>(mfg::AatArgs)") == ["aat_fused", "aat"]
    assert _c("k_rhs_tile<1, true, 0>(mfg::RhsArgs)",
              "k_rhs<false, false, true, 0>(mfg::RhsArgs)",
              "k_rhs_batch(mfg::RhsArgs const*, int const*, int)") == ["rhs", "apply_C",
                                                                       "rhs_batch"]
    assert _c("k_update(mfg::UpdArgs)") == ["update"]


def test_fused_preconditioner_passes():
    assert _c("k_tgemm_rows_fwd<1, 128, true>(a, b, c, int)",
              "k_cols_reg<float, 256>(mfg::ColsArgs<float>)",
              "k_rows_tgemm_inv<1, 128>(a, b, int, int)") == [
        "update_tgemm_rows_f32_fwd", "cols_solve_f32", "rows_tgemm_f32_inv"]
    assert _c("k_tgemm_rows_fwd<2, 64, false>(a, b, c, int)",
              "k_rows_tgemm_inv<3, 64>(a, b, int, int)") == ["tgemm_rows_f16_fwd",
                                                            "rows_tgemm_bf16_inv"]


def test_separate_preconditioner_kernels():
    got = _c("k_tgemm_lp<1, 128, 1, double, float, 8>(mfg::GemmArgs<double, float>)",
             "k_rows_reg<float, 256>(mfg::RowsArgs<float>)",
             "k_cols_reg<float, 256>(mfg::ColsArgs<float>)",
             "k_rows_reg<float, 256>(mfg::RowsArgs<float>)",
             "k_tgemm_lp<1, 128, 1, float, double, 8>(mfg::GemmArgs<float, double>)")
    assert got == ["tgemm_f32_fwd", "rows_fwd_f32", "cols_solve_f32", "rows_inv_f32",
                   "tgemm_f32_inv"]
