// dd_launch.h -- host-side interface of the kernels in dd_kernels.hip: plain
// argument structs and launcher functions used by the solver driver.
#pragma once

#include <hip/hip_runtime.h>

#include "dd_device.h"

namespace dd {

constexpr int BLAS_WG = 256;        // threads per workgroup of the vector kernels
constexpr int BLAS_MAX_WG = 4096;   // cap on their grid (grid-stride loops beyond it)
constexpr int GCR_MAX_NKV = 16;     // longest GCR cycle (vectors kept per restart)
constexpr int MAX_PARTIALS = BLAS_MAX_WG * 2 * GCR_MAX_NKV;
constexpr int MAX_BLOCK_VOLUME = 256;  // one SAP block per workgroup, one thread per site

// SAP half-sweep flags
constexpr int SAP_FIRST = 1;  // read s from the source b (s = b at the start of Alg. 1)
constexpr int SAP_PRE = 2;    // subtract the cross-block term A_{c c'} x_{c'} first
constexpr int SAP_TAIL = 4;   // tail of Alg. 1: produce x only, leave s alone
constexpr int SAP_FACES_OUT = 8;  // packed-FP16 half-sweep: leave face hop terms for the next half-sweep
// the fused tail of Alg. 3 (FP32 arithmetic): with TAIL also write this colour's rows of A x
constexpr int SAP_AMSAP = 16;      //   the in-block part A_cc x_c
constexpr int SAP_AMSAP_PRE = 32;  //   and the cross-block term of this launch, A_{c c'} x_{c'}
constexpr int SAP_CROSS_ONLY = 64; // only add A_{c c'} x_{c'} of the final x to those rows (Alg. 3, last step)

struct Phase4 {
    double re[4], im[4];
};

// sigma^pm_{mu nu}: the 2x2 diagonal blocks of P sigma_{mu nu} P for the six
// planes mu < nu, P = [[1, 1], [1, -1]] / sqrt 2 on the spin pairs
struct SigmaBlocks {
    double re[6][2][2][2];
    double im[6][2][2][2];
};

struct DiracArgs {
    void *out;
    const void *in;
    const void *links;
    const void *clover;  // 1 + C blocks (op D / D^dagger) or C_inv blocks (op A)
    int pin, pout, pg;   // precisions: 0 FP64, 1 FP32, 2 FP16
    int op;              // 0 D, 1 A, 2 D^dagger
    double kappa;
    Phase4 phase;
};

// the right-hand sides one packed-FP16 SAP launch sweeps, one after another in each workgroup:
// right-hand side idx[k] has its spinor fields sp_stride bytes and its face terms face_stride
// bytes after those of right-hand side 0 (n = 0: the single fields of the arguments)
constexpr int SAP_RHS_MAX = 16;
struct SapRhs {
    int n;
    int idx[SAP_RHS_MAX];
    long long sp_stride, face_stride;
};

struct SapArgs {
    const void *b;  // source (storage precision)
    void *s;        // work vector
    void *x;        // output M_SAP b
    const void *links;  // FP32 or FP16 links
    const void *cinv;   // FP32 or FP16 C_inv; the packed-FP16 half-sweep: the SAP-ready pair coefficients
    int prec;  // 1 FP32 storage, 2 FP16 storage
    int n_jac;
    double kappa;
    Phase4 phase;
    void *ax;     // FP32 arithmetic with SAP_AMSAP / SAP_CROSS_ONLY: A M_SAP b (storage precision)
    void *faces;  // packed-FP16 half-sweep: face hop terms (sap_face_bytes), written and read in turn
    SapRhs rhs;   // packed-FP16 half-sweep: the right-hand sides of a batch (n = 0: one)
};

enum BlasKind {
    BLAS_DOT = 0,
    BLAS_DOT_NORM,
    BLAS_NORM2,
    BLAS_UPDATE1,
    BLAS_UPDATE2,
    BLAS_PUPDATE,
    BLAS_AXPBY,
    BLAS_SUB_NORM,
    BLAS_CONVERT,
    BLAS_CINV_SRC,
    BLAS_UPDATE1_H,  // FP32 r -= c01 q ; |r|^2 ; v2 = r in FP16 storage (the next SAP input)
    BLAS_UPDATE2_MM, // FP32 y += c01 v1 + c23 v2 (FP16 v1, v2) ; r -= c23 t ; |r|^2, <rt|r>
    BLAS_PUPDATE_H,  // FP32 p = r + c01 (p - c23 q) ; v3 = p in FP16 storage
    BLAS_CAXPY,      // v0 += c01 v1 (FP32 v0, v1 at precision p1)
};

struct BlasArgs {
    int kind;
    void *v[6];
    int p[6];
    double c[4];
    double *partials;
};

// One launch of a vector kernel over several lattices (the lockstep multi-lattice
// solver): lattice k of the table runs the kernel's grid-stride loop over its own sites
// with nwg workgroups, launch workgroups item0 .. item0 + nwg - 1, its fields and
// coefficients as in BlasArgs, and leaves its partial sums at partials[poff + w nv + q].
// The table travels by value in the kernel arguments.
constexpr int MULTI_BLAS_MAX = 16;
struct MultiBlasLat {
    Geom g;
    void *v[6];
    double c[4];
    int item0, nwg;
    long long poff;
};
struct MultiBlasTab {
    MultiBlasLat e[MULTI_BLAS_MAX];
    int n;
};

constexpr int MRHS_FIRST_VECTOR = 8;  // batched-A variants from here on are vector kernels (FP16 inputs too)

// A = I - kappa C_inv H on a batch of FP32 internal-layout spinors (nrhs fields,
// one after another, 12 V complex apart), FP32 links and C_inv
struct MrhsArgs {
    const float2 *in;    // FP32 inputs (pin 1)
    const void *in16;    // FP16-storage inputs (pin 2): nrhs fields of 12 V half2 + V scales, one after another
    int pin;             // 1 or 2; FP16 inputs run the vector kernel only
    float2 *out;
    const float2 *u;     // FP32 links
    const float2 *cinv;  // FP32 C_inv blocks
    int nrhs;            // 1..12
    double kappa;
    Phase4 phase;
};

// one lattice of a multi-lattice launch: A = I - kappa C_inv H with FP32 links and
// C_inv, input at the launch's precision, FP32 output
struct LatDesc {
    Geom g;
    const void *in;
    void *out;
    const void *u;     // FP32 links
    const void *cinv;  // FP32 C_inv
    Phase4 phase;
    double kappa;
    int item0;  // first work item (256-site chunk) of this lattice
};

// one lattice of a multi-lattice packed-FP16 half-sweep (4^4 blocks, one right-hand side)
struct SapLat {
    Geom g;
    SpinorField<2> b, s, x;  // source, work vector, output (FP16 storage)
    const __half2 *u16;      // FP16 links (12 reals)
    const __half2 *cpsap;    // SAP-ready FP16 C_inv pair coefficients (launch_sap_prep)
    Phase4 ph;
    float kappa;
    int n_jac;
    __half2 *ft;  // face hop terms (sap_face_bytes)
    int item0;    // first work item of this lattice
};

constexpr int SAP_MULTI_MAX = 12;
struct SapLatTab {
    SapLat e[SAP_MULTI_MAX];
    int n;
};

struct ForceArgs {
    const void *psi, *chi;  // FP64 internal-layout spinors
    const void *u64;        // FP64 links
    const void *clov64;     // FP64 clover blocks 1 + C (dL/dc_SW when c_SW != 0)
    void *y;                // work: 54 complex per site (six planes of 3x3)
    void *out;              // canonical [4][Lt][Lz][Ly][Lx][3][3] complex double
    double *partials;       // per-workgroup partial sums of dL/dc_SW (nullptr: skip)
    double *dcsw;           // device scalar receiving dL/dc_SW
    SigmaBlocks sig;
    double kcsw, kappa, csw;
    Phase4 phase;
    int su3;  // 0: gradient W^dagger per link; 1: traceless Hermitian su(3) force
};

// sum of v over the workgroup (BLAS_WG threads): wavefront shuffles, then LDS;
// thread 0 writes the workgroup's partials[wid * NV + k]
template <int NV> DD_INL void wg_reduce_store_at(double (&v)[NV], double *partials, long long wid)
{
    __shared__ double red[NV][BLAS_WG / 64];
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[k][wave] = v[k];
    wg_barrier();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double t = 0;
            for (int q = 0; q < BLAS_WG / 64; ++q) t += red[k][q];
            partials[wid * NV + k] = t;
        }
}

// ... at partials[blockIdx.x * NV + k]
template <int NV> DD_INL void wg_reduce_store(double (&v)[NV], double *partials)
{
    wg_reduce_store_at<NV>(v, partials, blockIdx.x);
}

// canonical <-> internal spinor copies; g5 = true applies gamma_5 on the way
hipError_t launch_pack_spinor(const Geom &g, hipStream_t st, int prec, void *dst, const void *src, bool g5 = false);
hipError_t launch_unpack_spinor(const Geom &g, hipStream_t st, int prec, void *dst, const void *src, bool g5 = false);
hipError_t launch_pack_links(const Geom &g, hipStream_t st, const void *src, void *u64, void *u32, void *u16,
                             int *bad);
hipError_t launch_clover(const Geom &g, hipStream_t st, const void *u64, const SigmaBlocks &sig, double kcsw,
                         void *clov64, void *cinv32, void *cinv16, int *bad);
hipError_t launch_dirac(const Geom &g, hipStream_t st, const DiracArgs &a);
size_t sap_lds_bytes(const Geom &g, int prec);
hipError_t launch_sap_half(const Geom &g, hipStream_t st, const SapArgs &a, int colour, int flags);
// the same half-sweep with FP16 storage and packed FP16 block-local arithmetic; the cross-block
// term travels between half-sweeps as face hop terms (sap_face_bytes per lattice)
size_t sap_pk_lds_bytes(const Geom &g);
// the SAP-ready copy of C_inv the packed-FP16 half-sweep reads instead of the FP16 C_inv:
// its pair coefficients, 36 half2 per site
hipError_t launch_sap_prep(const Geom &g, hipStream_t st, const void *cinv16, void *cpsap);
size_t sap_face_bytes(const Geom &g);
hipError_t launch_sap_half_pk(const Geom &g, hipStream_t st, const SapArgs &a, int colour, int flags);
// the table entry of one lattice for the multi-lattice half-sweep, the work items of one
// lattice in it, and that launch: the nlat lattices of the table (host memory; it travels in
// the kernel arguments, SAP_MULTI_MAX lattices per launch) share the block shape of g
SapLat sap_lat(const Geom &g, const SapArgs &a, int item0);
int sap_multi_items(const Geom &g);
hipError_t launch_sap_half_pk_multi(const Geom &g, hipStream_t st, const SapLat *lat, int nlat, int colour,
                                    int flags);
int blas_grid(const Geom &g);
// grid of a grid-stride loop over the sites (one thread per site, at most BLAS_MAX_WG workgroups)
int blas_grid_sites(const Geom &g);
hipError_t launch_blas(const Geom &g, hipStream_t st, const BlasArgs &a);

// ---- flexible GCR: k directions p_j (FP16 storage) with images z_j (FP32)
struct VecSet {
    void *v[GCR_MAX_NKV];
    double re[GCR_MAX_NKV], im[GCR_MAX_NKV];
};
// <z_j | z> for j < k: 2k partial sums per workgroup; z_j and z FP32 (prec 1) or FP64 (prec 0)
hipError_t launch_multidot(const Geom &g, hipStream_t st, const VecSet &zs, int k, void *z, double *partials,
                           int prec = 1);
// flexible GMRES: w -= sum_j coef_j v_j (FP64, j < k), partial |w|^2; x (FP64) += sum_j coef_j z_j (FP32)
hipError_t launch_orth64(const Geom &g, hipStream_t st, const VecSet &vs, int k, void *w, double *partials);
hipError_t launch_multi_axpy64(const Geom &g, hipStream_t st, const VecSet &zs, int k, void *x);
// z -= sum_j coef_j z_j (j < k); partials: |z|^2, <z|r>
hipError_t launch_gcr_orth(const Geom &g, hipStream_t st, const VecSet &zs, int k, void *z, void *r,
                           double *partials);
// z *= 1/bn ; r -= c z ; partial |r|^2
hipError_t launch_gcr_rupdate(const Geom &g, hipStream_t st, void *z, void *r, double inv_bn, double cre, double cim,
                              double *partials);
// y (FP32) += sum_j coef_j p_j, p_j at precision pp (FP16 or FP32)
hipError_t launch_multi_axpy(const Geom &g, hipStream_t st, const VecSet &ps, int k, int pp, void *y);
hipError_t launch_finalize(hipStream_t st, const double *partials, int nwg, int nv, double *out);
// kind in {BLAS_DOT, BLAS_DOT_NORM, BLAS_UPDATE1_H, BLAS_UPDATE2_MM (FP16 M p, M r), BLAS_PUPDATE_H}
// on the lattices of t (total workgroups: the sum of their nwg)
hipError_t launch_blas_multi(hipStream_t st, int kind, const MultiBlasTab &t, int total, double *partials);
// out[3 slot[k] + q] = the fixed-order sum of lattice k's nv partials, for the lattices of t
hipError_t launch_finalize_multi(hipStream_t st, const MultiBlasTab &t, const int *slot, const double *partials, int nv,
                                 double *out);

// A on several lattices in one persistent launch (work queue over (lattice, chunk)
// items, desc_dev in device memory, counter: one device int, cleared here)
hipError_t launch_dirac_multi(hipStream_t st, const LatDesc *desc_dev, int nlat, int total, int pin, int *counter);

// multi right-hand-side A on the matrix cores; variant in [0, mrhs_variant_count())
int mrhs_variant_count();
const char *mrhs_variant_name(int v);
hipError_t launch_dirac_mrhs(const Geom &g, hipStream_t st, const MrhsArgs &a, int variant);

// fermion force of L = |D^{-1} phi|^2 from psi = D^{-1} phi and chi = D^{-dagger} psi
hipError_t launch_force(const Geom &g, hipStream_t st, const ForceArgs &a);

// the force's work field (54 complex doubles per site) in a fixed device array, for
// the entry point that allocates nothing: its size, and its address on the current
// device (looked up once per device)
constexpr size_t FORCE_SCRATCH_BYTES = (size_t)64 << 20;
constexpr int MAX_DEVICES = 64;
hipError_t force_scratch_address(void **ptr);

}  // namespace dd
