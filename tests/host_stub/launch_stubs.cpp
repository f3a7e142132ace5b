// Kernel launchers replaced by no-ops: the host driver and the server run on
// the CPU against hip/hip_runtime.h of this directory (host-logic test).
#include "rss_internal.h"
struct dim3s threadIdx, blockIdx, blockDim;
namespace rss {
template <class R> void launch_leaf_assemble(const Prob<R>*, int, int, int, hipStream_t) {}
template <class R> void launch_build_C(const Prob<R>*, const Phase<R>&, int, hipStream_t) {}
template <class R> void launch_cpqr(const Prob<R>*, const Phase<R>&, int, int, hipStream_t) {}
template <class R> int cpqr_mg_groups(int nbox, int, int) { return nbox < 8 ? 4 : 1; }
template <class R> int solve_group(int, int, int nrhs) { return nrhs < 16 ? nrhs : 16; }
template <class R> bool launch_cpqr_mg(const Prob<R>*, const Phase<R>&, int, int, int, double*, double*, unsigned*, int*, unsigned, hipStream_t) { return true; }
template <class R> void launch_sparsify(const Prob<R>*, const Phase<R>&, int, bool, hipStream_t) {}
int gram_tile_groups(int nmax) { return nmax > 64 ? 3 : 1; }
template <class R> void launch_gram(const Prob<R>*, const Phase<R>&, const GramWs&, int, hipStream_t) {}
template <class R> void launch_chol(const Prob<R>*, const Phase<R>&, const GramWs&, int, hipStream_t) {}
template <class R> void launch_inverse(const Prob<R>*, const Phase<R>&, int*, int, hipStream_t) {}
template <class R> void launch_plan_y(const Prob<R>*, const Phase<R>&, GemmDesc<R>*, hipStream_t) {}
template <class R> void launch_compact(const Prob<R>*, const Phase<R>&, int, hipStream_t) {}
template <class R> void launch_gemm(const GemmDesc<R>*, int, int, int, hipStream_t) {}
template <class R> void launch_schur(const Prob<R>*, const Phase<R>&, int, hipStream_t) {}
template <class R> void launch_assemble_pairs(const PairDesc*, int, const ListEntry*, int, int, const Prob<R>*, hipStream_t) {}
template <class R> void launch_root_inverse(const RootDesc<R>*, int, int, GemmDesc<R>*, int*, hipStream_t) {}
size_t root_work_elems(int n) { return (size_t)65 * n; }
template <class R> void launch_solve_fwd(const SolveProb<R>*, const Phase<R>&, int, int, int, int, SolveTile, cx<R>*, hipStream_t) {}
template <class R> size_t solve_work_elems(int nbox, int rmax, int S, int nrhs) { return (size_t)nbox * S * rmax * nrhs; }
template <class R> void launch_solve_bwd(const SolveProb<R>*, const Phase<R>&, int, int, int, int, SolveTile, cx<R>*, hipStream_t) {}
int solve_slices(int nbox, int) { return nbox < 64 ? 4 : 1; }
template <class R> bool solve_fused_fits(int, int rmax, int) { return rmax < 64; }
template <class R> void launch_root_apply(const RootApply<R>*, int, int, int, GemmDesc<R>*, hipStream_t) {}
#define I(R) \
template void launch_leaf_assemble<R>(const Prob<R>*, int, int, int, hipStream_t); \
template void launch_build_C<R>(const Prob<R>*, const Phase<R>&, int, hipStream_t); \
template void launch_cpqr<R>(const Prob<R>*, const Phase<R>&, int, int, hipStream_t); \
template void launch_sparsify<R>(const Prob<R>*, const Phase<R>&, int, bool, hipStream_t); \
template void launch_gram<R>(const Prob<R>*, const Phase<R>&, const GramWs&, int, hipStream_t); \
template void launch_chol<R>(const Prob<R>*, const Phase<R>&, const GramWs&, int, hipStream_t); \
template int cpqr_mg_groups<R>(int, int, int); \
template int solve_group<R>(int, int, int); \
template bool solve_fused_fits<R>(int, int, int); \
template bool launch_cpqr_mg<R>(const Prob<R>*, const Phase<R>&, int, int, int, double*, double*, unsigned*, int*, unsigned, hipStream_t); \
template void launch_inverse<R>(const Prob<R>*, const Phase<R>&, int*, int, hipStream_t); \
template void launch_plan_y<R>(const Prob<R>*, const Phase<R>&, GemmDesc<R>*, hipStream_t); \
template void launch_compact<R>(const Prob<R>*, const Phase<R>&, int, hipStream_t); \
template void launch_gemm<R>(const GemmDesc<R>*, int, int, int, hipStream_t); \
template void launch_schur<R>(const Prob<R>*, const Phase<R>&, int, hipStream_t); \
template void launch_assemble_pairs<R>(const PairDesc*, int, const ListEntry*, int, int, const Prob<R>*, hipStream_t); \
template void launch_root_inverse<R>(const RootDesc<R>*, int, int, GemmDesc<R>*, int*, hipStream_t); \
template void launch_solve_fwd<R>(const SolveProb<R>*, const Phase<R>&, int, int, int, int, SolveTile, cx<R>*, hipStream_t); \
template size_t solve_work_elems<R>(int, int, int, int); \
template void launch_solve_bwd<R>(const SolveProb<R>*, const Phase<R>&, int, int, int, int, SolveTile, cx<R>*, hipStream_t); \
template void launch_root_apply<R>(const RootApply<R>*, int, int, int, GemmDesc<R>*, hipStream_t);
I(double) I(float)
void launch_kernel_block(const KParams&, const double*, const int*, int64_t, const int*, int64_t, cx<double>*, hipStream_t) {}
void* residual_static_scratch() { return nullptr; }
void launch_grid_setup(const GridDesc&, cx<double>*, double*, cx<double>*, hipStream_t) {}
void launch_grid_apply(const GridDesc&, const cx<double>*, const cx<double>*, cx<double>*, int64_t, int, cx<double>*, int, hipStream_t) {}
void launch_cdot(const cx<double>*, const cx<double>*, int64_t, int nrhs, cx<double>*, cx<double>* out, hipStream_t) { for (int i = 0; i < nrhs; ++i) out[i] = cx<double>{1.0, 0.0}; }
void launch_caxpby(const cx<double>*, cx<double>*, int64_t, int, const cx<double>*, const cx<double>*, hipStream_t) {}
void launch_lincomb_sub(const cx<double>*, int64_t, int, const cx<double>*, cx<double>*, int64_t, int, hipStream_t) {}
int residual_slices(int64_t target_blocks) { return target_blocks >= 1024 ? 1 : 4; }
void launch_residual(const ResDesc*, const ResBlock*, int, const ResBlock*, int, int, hipStream_t) {}
void launch_colnorms(const cx<double>*, int64_t, int nrhs, double* out, hipStream_t) { for (int i = 0; i < nrhs; ++i) out[i] = 1.0; }
void launch_scale_to_c64(const cx<double>*, int64_t, int, const double*, cx<float>*, hipStream_t) {}
void launch_axpy_from_c64(const cx<float>*, int64_t, int, const double*, cx<double>*, hipStream_t) {}
void launch_cast_c64(const cx<double>*, int64_t, int, cx<float>*, hipStream_t) {}
void launch_fill_u64(unsigned long long*, int64_t, unsigned long long, hipStream_t) {}
void launch_add_c128(cx<double>*, const cx<double>*, int64_t, hipStream_t) {}
}
