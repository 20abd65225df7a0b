// C ABI of the solver: plan creation, transformed-kernel build, solves.
//
// The paper's boundary convention (section 2.2.2 and appendix A: device code
// in its own shared library behind bind(C) entry points that pass raw
// addresses, the caller keeping ownership and sharing by pointer rather than
// by copy) is kept: every entry point takes plain device pointers and sizes,
// validates them before any HIP call and reports a status code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "ps_internal.hpp"

namespace {

thread_local std::string g_last_error;

ps_status fail(ps_status s, const std::string& msg)
{
    g_last_error = msg;
    return s;
}

ps_status device_fail(hipError_t e, const char* where)
{
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return PS_ERR_DEVICE;
}

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// Solve records of a batch, kept in the workspace of the batch's first plan.
constexpr int MAX_BATCH = 1024;
size_t batch_bytes(int ns) { return align_up((size_t)ns * sizeof(ps::SolveRec)); }

bool is_plain(ps_precision p) { return p == PS_F64_PLAIN || p == PS_F32_PLAIN; }
bool is_f64(ps_precision p) { return p == PS_F64 || p == PS_F64_PLAIN; }

// cos and sin of 2 pi a / L for integers, with the angle reduced exactly to
// [0, pi/4] by quadrant and octant symmetry before the double libm call.
void unit_root(long a, long L, double& c, double& s)
{
    a %= L;
    if (a < 0) a += L;
    const long q = (4 * a) / L;       // quadrant
    const long t = 4 * a - q * L;     // angle within quadrant = (pi/2) t / L, t in [0, L)
    const double half_pi = 1.57079632679489661923;
    double c0, s0;
    if (2 * t <= L) {
        const double ang = half_pi * (double)t / (double)L;
        c0 = std::cos(ang);
        s0 = std::sin(ang);
    } else {
        const double ang = half_pi * (double)(L - t) / (double)L;
        c0 = std::sin(ang);
        s0 = std::cos(ang);
    }
    switch (q) {
    case 0: c = c0; s = s0; break;
    case 1: c = -s0; s = c0; break;
    case 2: c = -c0; s = -s0; break;
    default: c = s0; s = -c0; break;
    }
}

// Twiddle tables of a radix plan (stages >= 1), entry (q, m) =
// exp(-2 pi i q m / (NS R)) for q < R and residue m < NS: first every stage
// by rows (m major), then every stage by columns (q major), matching
// Radices::tw_off and tw_size on the device.
std::vector<std::complex<double>> plan_table(const std::vector<int>& rad)
{
    std::vector<std::complex<double>> rows, cols;
    long ns = rad.empty() ? 1 : rad[0];
    for (size_t s = 1; s < rad.size(); ++s) {
        const long r = rad[s];
        auto w = [&](long q, long m) {
            double c, sn;
            unit_root(q * m, ns * r, c, sn);
            return std::complex<double>(c, -sn);
        };
        for (long m = 0; m < ns; ++m)
            for (long q = 0; q < r; ++q) rows.push_back(w(q, m));
        for (long q = 0; q < r; ++q)
            for (long m = 0; m < ns; ++m) cols.push_back(w(q, m));
        ns *= r;
    }
    rows.insert(rows.end(), cols.begin(), cols.end());
    return rows;
}

// Round a double to the nearest bf16 value (8 significant bits, ties to even).
double bf16_round(double a)
{
    if (a == 0.0 || !std::isfinite(a)) return a;
    int e;
    const double m = std::frexp(a, &e);  // a = m 2^e, 0.5 <= |m| < 1
    return std::ldexp(std::nearbyint(std::ldexp(m, 8)), e - 8);
}

unsigned short bf16_bits(double v)  // v already a bf16 value
{
    const float f = (float)v;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return (unsigned short)(u >> 16);
}

// Matrix pieces of the split-bf16 DFT-16 in the lane layout of
// v_mfma_f32_32x32x16_bf16's A operand: [piece][K chunk][lane][8].  Row m of
// the operand is row perm(m) of the real 32x32 forward DFT-16 matrix
// [[Wr, -Wi], [Wi, Wr]], perm(8j + 4h + i) = 16 (j / 2) + 8 h + 4 (j % 2) + i,
// so that a lane's accumulator holds the outputs whose inputs it held.
std::vector<unsigned short> split_dft16_table()
{
    double M[32][32];
    for (int a = 0; a < 16; ++a)
        for (int b = 0; b < 16; ++b) {
            double c, sn;
            unit_root((long)a * b, 16, c, sn);
            const double wr = c, wi = -sn;  // exp(-2 pi i ab / 16)
            M[a][b] = wr;
            M[a][16 + b] = -wi;
            M[16 + a][b] = wi;
            M[16 + a][16 + b] = wr;
        }
    std::vector<unsigned short> t(3 * 2 * 64 * 8);
    for (int chunk = 0; chunk < 2; ++chunk)
        for (int lane = 0; lane < 64; ++lane)
            for (int i = 0; i < 8; ++i) {
                const int m = lane % 32, kk = 8 * (lane / 32) + i;
                const int j = m / 8, hh = (m / 4) % 2, ii = m % 4;
                const int row = 16 * (j / 2) + 8 * hh + 4 * (j % 2) + ii;
                const double v = M[row][16 * chunk + kk];
                const double p0 = bf16_round(v);
                const double r1 = v - p0;
                const double p1 = bf16_round(r1);
                const double p2 = bf16_round(r1 - p1);
                const double pc[3] = {p0, p1, p2};
                for (int piece = 0; piece < 3; ++piece)
                    t[((piece * 2 + chunk) * 64 + lane) * 8 + i] = bf16_bits(pc[piece]);
            }
    return t;
}

template <typename T> void append_table(std::vector<unsigned char>& blob, size_t& off,
                                        const std::vector<std::complex<double>>& t)
{
    off = align_up(blob.size());
    blob.resize(off + std::max<size_t>(1, t.size()) * 2 * sizeof(T), 0);
    T* d = reinterpret_cast<T*>(blob.data() + off);
    for (size_t i = 0; i < t.size(); ++i) {
        d[2 * i] = (T)t[i].real();
        d[2 * i + 1] = (T)t[i].imag();
    }
}

// P = 2n = 16 m with 1 <= m <= 64 and no prime factor of m above 5 (the
// lengths the radix plans cover).
bool supported_n(int n)
{
    if (n < 8 || n > 512 || n % 8 != 0) return false;
    int m = n / 8;
    for (int f : {2, 3, 5})
        while (m % f == 0) m /= f;
    return m == 1;
}

// K(0) for cells of spacings dx, dy, dz: -self_coeff/dx for a cube; for a
// box, the box's average of 1/|r| scaled by self_coeff over the unit cube's
// average 3 ln(2 + sqrt 3) - pi/2 (so that the two agree on cubes).  The
// average over the box [-a,a] x [-b,b] x [-c,c] is 8 F(a, b, c) / (8abc)
// with F the integral of 1/|r| over [0,a] x [0,b] x [0,c]:
//   F = bc asinh(a/sqrt(b^2+c^2)) + ca asinh(b/sqrt(c^2+a^2)) + ab asinh(c/sqrt(a^2+b^2))
//       - (a^2 atan(bc/(a r)) + b^2 atan(ca/(b r)) + c^2 atan(ab/(c r))) / 2,  r = |(a, b, c)|.
double self_value(double dx, double dy, double dz, double self_coeff)
{
    if (dx == dy && dy == dz) return -self_coeff / dx;
    const double a = 0.5 * dx, b = 0.5 * dy, c = 0.5 * dz, r = std::sqrt(a * a + b * b + c * c);
    const double f = b * c * std::asinh(a / std::hypot(b, c)) + c * a * std::asinh(b / std::hypot(c, a)) +
                     a * b * std::asinh(c / std::hypot(a, b)) -
                     0.5 * (a * a * std::atan(b * c / (a * r)) + b * b * std::atan(c * a / (b * r)) +
                            c * c * std::atan(a * b / (c * r)));
    const double average = f / (a * b * c);
    const double unit_cube = 3.0 * std::log(2.0 + std::sqrt(3.0)) - 2.0 * std::atan(1.0);
    return -self_coeff / unit_cube * average;
}

bool capturing(hipStream_t s, bool& cap, hipError_t& err)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    err = hipStreamIsCapturing(s, &st);
    cap = st != hipStreamCaptureStatusNone;
    return err == hipSuccess;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

}  // namespace

struct ps_plan_s {
    int n = 0, P = 0, H = 0;              // x axis (every axis of a cube)
    int nx = 0, ny = 0, nz = 0;           // cells per axis
    bool box = false;                     // axes of unequal length: the kernels built for boxes
    double dx = 0.0, dy = 0.0, dz = 0.0;  // cell spacings along x, y, z
    ps_precision prec = PS_F64;
    size_t real_bytes = 0;
    std::vector<int> radices;             // forward radix plan of the x axis
    // workspace layout (byte offsets)
    std::vector<unsigned char> tables;
    size_t off_tab = 0, tab_bytes = 0;
    // offsets inside the table blob, per axis (x, y, z; equal axes share tables)
    size_t tw_f[3] = {}, tw_i[3] = {}, tw_f64[3] = {};
    size_t tw_f1[3] = {}, tw_i1[3] = {};  // family-1 plan tables
    size_t split_tab = 0;                   // split-bf16 DFT-16 matrix pieces
    ps::PrunedVariant var;                  // kernel variant per pass
    size_t off_ghat = 0, ghat_bytes = 0;
    size_t off_t1 = 0, off_t2 = 0, off_t3 = 0;  // pruned intermediates
    size_t off_pad = 0, off_spec = 0;       // plain intermediates
    size_t off_gscr = 0;                    // kernel-build scratch (aliases intermediates)
    size_t off_rec = 0;                     // this plan's own solve record (pruned plans)
    size_t off_batch = 0;                   // solve records of a batch this plan leads
    size_t ws_bytes = 0;
    std::vector<uintptr_t> batch_sig;       // batch whose records are in the workspace
    // streams and events that run a led batch's groups side by side
    std::vector<hipStream_t> aux;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;
    // copy streams and events of host-resident solves (fork, upload, solve, download x 2 slots)
    hipStream_t up = nullptr, down = nullptr;
    hipEvent_t hev[7] = {};
    // bound state
    unsigned char* ws = nullptr;
    bool ready = false;
    double G = 1.0, self_coeff = 2.38;

    ~ps_plan_s()
    {
        for (hipStream_t s : aux) (void)hipStreamDestroy(s);
        for (hipEvent_t e : join) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        if (up) (void)hipStreamDestroy(up);
        if (down) (void)hipStreamDestroy(down);
        for (hipEvent_t e : hev)
            if (e) (void)hipEventDestroy(e);
    }
};

namespace {

ps_status check_plan(ps_plan p)
{
    if (!p) return fail(PS_ERR_INVALID, "plan is NULL");
    return PS_OK;
}

size_t cells(ps_plan p) { return (size_t)p->nx * p->ny * p->nz; }
int axis_pad(ps_plan p, int axis) { return 2 * (axis == 0 ? p->nx : axis == 1 ? p->ny : p->nz); }

ps::SolveRec solve_rec(ps_plan p, const void* rho, void* phi)
{
    ps::SolveRec r{};
    r.rho = rho;
    r.phi = phi;
    r.t1 = p->ws + p->off_t1;
    r.t2 = p->ws + p->off_t2;
    r.t3 = p->ws + p->off_t3;
    r.ghat = p->ws + p->off_ghat;
    for (int a = 0; a < 3; ++a) {
        r.twf[a] = p->ws + p->off_tab + p->tw_f[a];
        r.twi[a] = p->ws + p->off_tab + p->tw_i[a];
        r.twf1[a] = p->ws + p->off_tab + p->tw_f1[a];
        r.twi1[a] = p->ws + p->off_tab + p->tw_i1[a];
    }
    r.nx = p->nx;
    r.ny = p->ny;
    r.nz = p->nz;
    return r;
}

// One solve with the plan's own record; rho and phi replace the input of
// pass 0 and the output of pass 4.
ps::PrunedBufs pruned_bufs(ps_plan p, const void* rho, void* phi, hipStream_t s)
{
    ps::PrunedBufs b;
    b.list = reinterpret_cast<const ps::SolveRec*>(p->ws + p->off_rec);
    b.count = 1;
    b.in[0] = rho;
    b.out[4] = phi;
    b.stab = reinterpret_cast<const unsigned short*>(p->ws + p->off_tab + p->split_tab);
    b.var = p->var;
    b.stream = s;
    b.px = axis_pad(p, 0);
    b.py = axis_pad(p, 1);
    b.pz = axis_pad(p, 2);
    b.box = p->box;
    b.nx = p->nx;
    b.ny = p->ny;
    b.nz = p->nz;
    return b;
}

hipError_t run_pruned(ps_precision prec, int lo, int hi, const ps::PrunedBufs& b);

// The kernels of one solve, enqueued on `st` (arguments already checked).
hipError_t enqueue_solve(ps_plan p, const void* d_rho, void* d_phi, hipStream_t st)
{
    if (is_plain(p->prec)) {
        ps::PlainBufs b;
        b.rho = d_rho;
        b.phi = d_phi;
        b.pad = p->ws + p->off_pad;
        b.spec = p->ws + p->off_spec;
        b.ghat = p->ws + p->off_ghat;
        b.twf = p->ws + p->off_tab + p->tw_f[0];
        b.twi = p->ws + p->off_tab + p->tw_i[0];
        b.stream = st;
        return is_f64(p->prec) ? ps::plain_run_f64(p->P, b) : ps::plain_run_f32(p->P, b);
    }
    const ps::PrunedBufs b = pruned_bufs(p, d_rho, d_phi, st);
    return run_pruned(p->prec, 0, 5, b);
}

// Device staging for host-resident solves: two input and two output slots.
size_t host_stage_bytes(ps_plan p) { return 4 * align_up(cells(p) * p->real_bytes); }

const char* prec_name(ps_precision p)
{
    switch (p) {
    case PS_F64: return "f64";
    case PS_F32: return "f32";
    case PS_F32_SPLIT: return "f32_split";
    case PS_F64_PLAIN: return "f64_plain";
    case PS_F32_PLAIN: return "f32_plain";
    }
    return "?";
}

// pass 6 (z tile): 2 values; x passes: family bit + 2 x rows selector (16, 8, 32 rows);
// y passes: family bit + 2 x persistent bit, or 4 + family bit (half tile)
int num_variants(int pass) { return pass == 2 ? ps::NUM_ZMODES : (pass == 1 || pass == 3) ? 8 : 6; }

// Whether variant v of a pass runs the radix-32-based plan family.
bool variant_needs_family1(int pass, int v)
{
    return pass == 6 ? false : pass == 2 ? (v == 2 || v == 5) : (v & 1) != 0;
}
// Whether the axis a pass transforms has the radix-32-based family.
bool family1_available(ps_plan p, int pass)
{
    const int axis = pass == 2 ? 2 : (pass == 1 || pass == 3) ? 1 : 0;
    return ps::has_family1(axis_pad(p, axis)) && p->prec != PS_F32_SPLIT;
}

// Runs passes [lo, hi) of a pruned plan's pipeline with its arithmetic.
hipError_t run_pruned(ps_precision prec, int lo, int hi, const ps::PrunedBufs& b)
{
    if (prec == PS_F64) return ps::pruned_run_f64(lo, hi, b);
    if (prec == PS_F32_SPLIT) return b.var.mterms == 3 ? ps::pruned_run_split3(lo, hi, b)
                                                       : ps::pruned_run_split6(lo, hi, b);
    return ps::pruned_run_f32(lo, hi, b);
}

int* variant_slot(ps::PrunedVariant& v, int pass)
{
    switch (pass) {
    case 0: return &v.x_fam;
    case 1: return &v.y_fam;
    case 2: return &v.zmode;
    case 3: return &v.yi_fam;
    case 6: return &v.ztile;
    default: return &v.xc_fam;
    }
}

// LDS row pitch of a length-P pencil (complex elements of eb bytes) whose
// plan starts with radix r0: the device engine's pad_pitch.
int lds_pitch(int P, int r0, int eb)
{
    const int G = r0 == 32 ? 32 : 16;
    const int lp = P + P / G + 1;
    return eb == 16 ? lp + (12 - lp % 8) % 8 : lp;
}

// Whether both x passes with `rows` rows per workgroup fit the 160 KB of LDS
// (the launchers' x_fits).
bool x_rows_fit(ps_plan p, int rows, bool fam1)
{
    const int P = axis_pad(p, 0), H = P / 2 + 1, eb = 2 * (int)p->real_bytes;
    std::vector<int> fwd;
    if (!ps::host_radices(P, fwd, fam1 ? 1 : 0) || fwd.empty()) return false;
    const int lf = (rows / 2) * lds_pitch(P, fwd.front(), eb);
    const int li = std::max((rows / 2) * lds_pitch(P, fwd.back(), eb), rows * (H + 1));  // inverse plan reversed
    return std::max(lf, li) * eb <= 160 * 1024;
}

// Whether `variant` is a kernel variant of `pass` that this plan can run.
bool variant_ok(ps_plan p, int pass, int variant)
{
    if (variant < 0 || variant >= num_variants(pass)) return false;
    if (variant_needs_family1(pass, variant) && !family1_available(p, pass)) return false;
    if (pass == 0 || pass == 4) {
        static const int ROWS[3] = {16, 8, 32};
        if ((variant >> 1) != 0 && p->box) return false;  // boxes: 16 rows per x tile
        if (!x_rows_fit(p, ROWS[variant >> 1], (variant & 1) && family1_available(p, pass))) return false;
    }
    // boxes run the one-tile-per-workgroup kernels only
    if (p->box && (pass == 1 || pass == 3) && (variant & 6)) return false;
    if (p->box && pass == 2 && variant >= 3) return false;
    // half-LDS z exchange: FP64 and FP32 cubes with P >= 512 (where the LDS
    // rows otherwise bound the pencils resident per compute unit)
    if (pass == 2 && variant >= 5 && ((p->prec != PS_F64 && p->prec != PS_F32) || axis_pad(p, 2) < 512)) return false;
    // half-LDS y exchanges (6, 7): the same plans
    if ((pass == 1 || pass == 3) && variant >= 6 && ((p->prec != PS_F64 && p->prec != PS_F32) || axis_pad(p, 1) < 512))
        return false;
    return true;
}

// Default z pass per padded length: the fastest form (variant 0..5) and
// tile width (0: full, 1: half), and for P > 256 the x passes' variants
// (family and rows per workgroup; 8 rows won for most FP64 lengths and for
// the inverse x pass of most FP32 lengths) and the y passes' (family,
// persistent form or half tile), measured on MI355X for FP64, FP32 and
// FP32-split.  P = 64, 96, 128, 192, 256 (the lengths of batches of uneven
// small solves): the wave-owned form on the full tile, the fastest for the
// 96-solve batch as a whole (groups run side by side on forked streams,
// where persistent forms, which fill the device, and the half tile measured
// 1-8% slower), though not always for one solve alone.  Other lengths: the
// pass timed alone on one cube of P/2 cells, each form at both widths; a
// choice replaced the earlier rule only where it was at least 3% faster.
struct ZDefault {
    int P;
    signed char zmode[3], ztile[3];  // [FP64, FP32, FP32-split]
    signed char x[3], xc[3];         // x_r2c and x_c2r variants; -1: the family rule
    signed char y[3], yi[3];         // forward and inverse y-pass variants; -1: the family rule
};
const ZDefault Z_DEFAULTS[] = {
    {  16, {1, 3, 1}, {0, 1, 0}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}},
    {  32, {1, 1, 1}, {0, 0, 0}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}},
    {  48, {1, 1, 0}, {0, 0, 1}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}},
    {  64, {1, 1, 1}, {0, 0, 0}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}},
    {  80, {1, 1, 0}, {0, 0, 1}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}},
    {  96, {1, 1, 1}, {0, 0, 0}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}},
    { 128, {1, 1, 1}, {0, 0, 0}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}},
    { 144, {2, 2, 1}, {1, 0, 0}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}},
    { 160, {1, 0, 0}, {0, 1, 0}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}},
    { 192, {1, 1, 1}, {0, 0, 0}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}},
    { 240, {1, 1, 4}, {1, 1, 1}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}},
    { 256, {1, 1, 1}, {0, 0, 0}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}},
    { 288, {0, 0, 1}, {0, 1, 1}, {2, 2, 4}, {1, 2, 4}, {-1, 5, -1}, {5, 5, -1}},
    { 320, {0, 0, 0}, {0, 1, 1}, {2, 2, -1}, {-1, -1, -1}, {-1, 4, -1}, {-1, 4, -1}},
    { 384, {0, 0, 0}, {0, 1, 1}, {-1, -1, -1}, {2, -1, -1}, {-1, -1, -1}, {-1, 4, -1}},
    { 400, {3, 3, 1}, {1, 0, 0}, {2, 3, 2}, {3, 3, -1}, {-1, 5, -1}, {1, 1, -1}},
    { 432, {3, 3, 1}, {0, 0, 0}, {1, 3, -1}, {3, 3, -1}, {1, 5, -1}, {1, 1, -1}},
    { 480, {3, 2, 1}, {1, 1, 1}, {-1, -1, -1}, {2, 2, 2}, {-1, 2, -1}, {-1, 5, -1}},
    { 512, {5, 3, 4}, {0, 0, 1}, {2, -1, -1}, {2, -1, -1}, {-1, 6, -1}, {-1, -1, 4}},
    { 576, {2, 2, 1}, {0, 0, 0}, {2, 1, -1}, {2, 1, 2}, {1, 7, 4}, {1, 7, -1}},
    { 640, {5, 5, 1}, {1, 0, 1}, {2, 1, -1}, {2, 2, 2}, {7, 7, 2}, {7, 7, 4}},
    { 720, {5, 2, 1}, {1, 1, 0}, {2, 1, -1}, {2, 2, 2}, {7, 7, 4}, {7, 7, 4}},
    { 768, {0, 5, 1}, {1, 0, 1}, {2, -1, -1}, {2, 2, 2}, {-1, 7, -1}, {7, 7, 4}},
    { 800, {5, 5, 1}, {1, 1, 0}, {2, 1, -1}, {2, 3, 2}, {1, 7, -1}, {7, 7, 4}},
    { 864, {5, 5, 1}, {1, 0, 0}, {3, 1, -1}, {3, 3, 2}, {1, 7, -1}, {7, 7, 4}},
    { 960, {5, 5, 1}, {1, 1, 0}, {2, -1, -1}, {2, 3, -1}, {1, 1, -1}, {6, 7, 4}},
    {1024, {5, 3, 1}, {0, 0, 1}, {2, -1, -1}, {2, 2, -1}, {-1, 7, -1}, {-1, -1, 4}},
};

// The measured defaults of length P, and the precision's column in them.
const ZDefault* measured_default(int P, ps_precision prec, int& k)
{
    k = prec == PS_F64 ? 0 : prec == PS_F32 ? 1 : prec == PS_F32_SPLIT ? 2 : -1;
    if (k < 0) return nullptr;
    for (const ZDefault& d : Z_DEFAULTS)
        if (d.P == P) return &d;
    return nullptr;
}

// Tuning cache: one line per (P, precision): "P prec x y z yi xc zt" (zt,
// the z-pass tile, may be absent: 0).  A line whose variants this plan
// cannot run is ignored; the split product-term count (not part of the
// line) is kept.
bool read_tuning(const char* path, ps_plan p)
{
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        int pp;
        std::string pr;
        int v[5], zt = 0;
        if (!(is >> pp >> pr >> v[0] >> v[1] >> v[2] >> v[3] >> v[4])) continue;
        if (!(is >> zt)) zt = 0;
        if (pp != p->P || pr != prec_name(p->prec)) continue;
        bool ok = zt == 0 || zt == 1;
        for (int k = 0; k < 5; ++k) ok = ok && variant_ok(p, k, v[k]);
        if (!ok) continue;
        for (int k = 0; k < 5; ++k) *variant_slot(p->var, k) = v[k];  // the last valid matching line wins
        p->var.ztile = zt;
        found = true;
    }
    return found;
}

bool write_tuning(const char* path, int P, ps_precision prec, const ps::PrunedVariant& v)
{
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (f && std::getline(f, line)) {
            std::istringstream is(line);
            int pp;
            std::string pr;
            if ((is >> pp >> pr) && pp == P && pr == prec_name(prec)) continue;
            if (!line.empty()) keep.push_back(line);
        }
    }
    std::ofstream o(path, std::ios::trunc);
    if (!o) return false;
    for (auto& l : keep) o << l << "\n";
    o << P << " " << prec_name(prec) << " " << v.x_fam << " " << v.y_fam << " " << v.zmode << " " << v.yi_fam << " "
      << v.xc_fam << " " << v.ztile << "\n";
    return (bool)o;
}

}  // namespace

extern "C" {

const char* ps_status_str(ps_status s)
{
    switch (s) {
    case PS_OK: return "ok";
    case PS_ERR_INVALID: return "invalid argument";
    case PS_ERR_UNSUPPORTED: return "unsupported size or precision";
    case PS_ERR_NOT_READY: return "plan has no built transformed kernel";
    case PS_ERR_DEVICE: return "HIP device error";
    case PS_ERR_CAPTURE: return "not allowed under stream capture";
    }
    return "unknown status";
}

const char* ps_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace {

// A plan for nx x ny x nz cells of spacings dx, dy, dz (a cube when the
// three lengths agree).
ps_status create_plan(ps_plan* out, int nx, int ny, int nz, double dx, double dy, double dz, ps_precision prec,
                      const char* tune_cache)
{
    if (!out) return fail(PS_ERR_INVALID, "out is NULL");
    *out = nullptr;
    for (double d : {dx, dy, dz})
        if (!(d > 0.0) || !std::isfinite(d)) return fail(PS_ERR_INVALID, "cell spacings must be positive and finite");
    if ((int)prec < (int)PS_F64 || (int)prec > (int)PS_F32_PLAIN)
        return fail(PS_ERR_INVALID, "unknown precision " + std::to_string((int)prec));
    for (int n : {nx, ny, nz}) {
        if (n <= 0) return fail(PS_ERR_INVALID, "cell counts must be positive");
        if (!supported_n(n))
            return fail(PS_ERR_UNSUPPORTED,
                        "n = " + std::to_string(n) +
                            " unsupported (2n must be 16 m <= 1024 with m having no prime factor above 5)");
    }
    const bool box = !(nx == ny && ny == nz);
    if (box && is_plain(prec)) return fail(PS_ERR_UNSUPPORTED, "the plain method is built for cubes only");
    ps_plan p = new (std::nothrow) ps_plan_s();
    if (!p) return fail(PS_ERR_INVALID, "out of host memory");
    p->n = nx;
    p->P = 2 * nx;
    p->H = nx + 1;
    p->nx = nx;
    p->ny = ny;
    p->nz = nz;
    p->box = box;
    p->dx = dx;
    p->dy = dy;
    p->dz = dz;
    p->prec = prec;
    p->real_bytes = is_f64(prec) ? 8 : 4;
    if (!ps::host_radices(p->P, p->radices)) {
        delete p;
        return fail(PS_ERR_UNSUPPORTED, "no radix plan");
    }
    // twiddle tables per distinct axis length
    for (int a = 0; a < 3; ++a) {
        const int Pa = axis_pad(p, a);
        int same = -1;
        for (int b = 0; b < a && same < 0; ++b)
            if (axis_pad(p, b) == Pa) same = b;
        if (same >= 0) {
            p->tw_f[a] = p->tw_f[same];
            p->tw_i[a] = p->tw_i[same];
            p->tw_f1[a] = p->tw_f1[same];
            p->tw_i1[a] = p->tw_i1[same];
            p->tw_f64[a] = p->tw_f64[same];
            continue;
        }
        std::vector<int> fwd, fwd1;
        ps::host_radices(Pa, fwd);
        ps::host_radices(Pa, fwd1, 1);
        const std::vector<int> inv(fwd.rbegin(), fwd.rend()), inv1(fwd1.rbegin(), fwd1.rend());
        const auto tf = plan_table(fwd), ti = plan_table(inv), tf1 = plan_table(fwd1), ti1 = plan_table(inv1);
        if (is_f64(prec)) {
            append_table<double>(p->tables, p->tw_f[a], tf);
            append_table<double>(p->tables, p->tw_i[a], ti);
            append_table<double>(p->tables, p->tw_f1[a], tf1);
            append_table<double>(p->tables, p->tw_i1[a], ti1);
            p->tw_f64[a] = p->tw_f[a];
        } else {
            append_table<float>(p->tables, p->tw_f[a], tf);
            append_table<float>(p->tables, p->tw_i[a], ti);
            append_table<float>(p->tables, p->tw_f1[a], tf1);
            append_table<float>(p->tables, p->tw_i1[a], ti1);
            append_table<double>(p->tables, p->tw_f64[a], tf);
        }
    }
    if (prec == PS_F32_SPLIT) {
        const auto st = split_dft16_table();
        p->split_tab = align_up(p->tables.size());
        p->tables.resize(p->split_tab + st.size() * sizeof(unsigned short), 0);
        std::memcpy(p->tables.data() + p->split_tab, st.data(), st.size() * sizeof(unsigned short));
    }
    // Default variants, as measured fastest per pass on MI355X: where the
    // radix-32-based family exists (P = 512, 1024) it wins for the forward y
    // pass, while the x passes keep the radix-16-based family (except FP64
    // at P = 1024, whose forward x pass is faster on radix 32); at P = 1024
    // the inverse y pass runs persistent (radix-32 family in FP32, radix-16
    // in FP64).  Split plans keep the radix-16 stages (their matrix-core
    // DFT-16).  The z pass's form and tile width come from the measured
    // table Z_DEFAULTS (the rules below are its fallback).  Boxes take the
    // one-tile-per-workgroup forms, per axis length.
    const int Py = axis_pad(p, 1), Pz = axis_pad(p, 2);
    if (prec == PS_F32_SPLIT) {
        p->var.zmode = 1;
        p->var.mterms = 6;
    } else if (box) {
        p->var.y_fam = (Py == 512 || Py == 1024) ? 1 : 0;
        p->var.zmode = (Pz == 512 || Pz == 1024) && !(prec == PS_F64 && Pz >= 1024) ? 2 : 1;
    } else if (p->P == 512 || p->P == 1024) {
        p->var.y_fam = 1;
        p->var.zmode = prec == PS_F64 ? (p->P >= 1024 ? 1 : 2) : 3;
        if (p->P >= 1024) p->var.yi_fam = prec == PS_F64 ? 2 : 3;  // persistent inverse y pass
        if (p->P >= 1024 && prec == PS_F64) p->var.x_fam = 1;
    } else {
        p->var.zmode = 1;
    }
    // the z pass's form and tile width per length, as measured (boxes take
    // the one-tile-per-workgroup forms only), and the x passes' rows per
    // workgroup where the table has them (cubes)
    if (!is_plain(prec)) {
        int k = 0;
        const ZDefault* d = measured_default(Pz, prec, k);
        if (d && (!box || d->zmode[k] <= 2)) {
            p->var.zmode = d->zmode[k];
            p->var.ztile = d->ztile[k];
        }
        d = box ? nullptr : measured_default(p->P, prec, k);
        if (d && d->x[k] >= 0 && variant_ok(p, 0, d->x[k])) p->var.x_fam = d->x[k];
        if (d && d->xc[k] >= 0 && variant_ok(p, 4, d->xc[k])) p->var.xc_fam = d->xc[k];
        if (d && d->y[k] >= 0 && variant_ok(p, 1, d->y[k])) p->var.y_fam = d->y[k];
        if (d && d->yi[k] >= 0 && variant_ok(p, 3, d->yi[k])) p->var.yi_fam = d->yi[k];
    }
    if (tune_cache && !is_plain(prec) && !box) read_tuning(tune_cache, p);
    const size_t Ny = ny, Nz = nz, Hx = nx + 1, Hy = ny + 1, Hz = nz + 1;
    const size_t r = p->real_bytes, c = 2 * r;
    size_t off = 0;
    p->off_tab = off;
    p->tab_bytes = align_up(p->tables.size());
    off += p->tab_bytes;
    p->off_ghat = off;
    p->ghat_bytes = Hx * Hy * Hz * r;
    off += align_up(p->ghat_bytes);
    const size_t gscr = Hx * Hy * Hz * 8;
    if (is_plain(prec)) {
        const size_t P = p->P, H = p->H;
        p->off_pad = off;
        off += align_up(P * P * P * r);
        p->off_spec = off;
        const size_t spec = P * P * H * c;
        off += align_up(std::max(spec, gscr));
        p->off_gscr = p->off_spec;
    } else {
        p->off_t1 = off;
        const size_t hp = (Hx + 15) / 16 * 16;
        const size_t t1 = std::max(Hx, hp) * Nz * Ny * c, t2 = Hx * (2 * Ny) * Nz * c;
        off += align_up(t1);
        p->off_t2 = off;
        off += align_up(t2);
        p->off_t3 = off;
        off += align_up(t2);
        p->off_gscr = p->off_t1;
        if (p->off_gscr + gscr > off) off = align_up(p->off_gscr + gscr);
        p->off_rec = off;
        off += align_up(sizeof(ps::SolveRec));
        p->off_batch = off;
        off += batch_bytes(MAX_BATCH);
    }
    p->ws_bytes = off;
    *out = p;
    return PS_OK;
}

}  // namespace

extern "C" {

ps_status ps_plan_create(ps_plan* out, int n, double dx, ps_precision prec, const char* tune_cache)
{
    return create_plan(out, n, n, n, dx, dx, dx, prec, tune_cache);
}

ps_status ps_plan_create_box(ps_plan* out, int nx, int ny, int nz, double dx, double dy, double dz,
                             ps_precision prec, const char* tune_cache)
{
    return create_plan(out, nx, ny, nz, dx, dy, dz, prec, tune_cache);
}

ps_status ps_plan_workspace_bytes(ps_plan p, size_t* bytes)
{
    if (ps_status s = check_plan(p)) return s;
    if (!bytes) return fail(PS_ERR_INVALID, "bytes is NULL");
    *bytes = p->ws_bytes;
    return PS_OK;
}

ps_status ps_plan_query(ps_plan p, ps_plan_info* info)
{
    if (ps_status s = check_plan(p)) return s;
    if (!info) return fail(PS_ERR_INVALID, "info is NULL");
    std::memset(info, 0, sizeof(*info));
    info->n = p->n;
    info->p = p->P;
    info->h = p->H;
    info->precision = (int)p->prec;
    info->dx = p->dx;
    info->dy = p->dy;
    info->dz = p->dz;
    info->workspace_bytes = p->ws_bytes;
    info->ghat_bytes = p->ghat_bytes;
    info->ready = p->ready ? 1 : 0;
    info->nx = p->nx;
    info->ny = p->ny;
    info->nz = p->nz;
    for (size_t i = 0; i < p->radices.size() && i < 7; ++i) info->radices[i] = p->radices[i];
    if (!is_plain(p->prec)) {
        info->t1_offset = p->off_t1;
        info->t2_offset = p->off_t2;
        info->t3_offset = p->off_t3;
        for (int k = 0; k < 5; ++k) info->variant[k] = *variant_slot(p->var, k);
        info->split_terms = p->var.mterms;
        info->z_tile = p->var.ztile;
    }
    return PS_OK;
}

void ps_plan_destroy(ps_plan p) { delete p; }

ps_status ps_green_build(ps_plan p, void* d_workspace, double G, double self_coeff, void* stream)
{
    if (ps_status s = check_plan(p)) return s;
    if (!d_workspace) return fail(PS_ERR_INVALID, "workspace is NULL");
    if ((uintptr_t)d_workspace % ALIGN) return fail(PS_ERR_INVALID, "workspace must be 256-byte aligned");
    if (!std::isfinite(G) || !std::isfinite(self_coeff)) return fail(PS_ERR_INVALID, "G and self_coeff must be finite");
    hipStream_t st = (hipStream_t)stream;
    bool cap = false;
    hipError_t e;
    if (!capturing(st, cap, e)) return device_fail(e, "hipStreamIsCapturing");
    if (cap) return fail(PS_ERR_CAPTURE, "ps_green_build cannot run under stream capture");
    p->ready = false;
    unsigned char* ws = static_cast<unsigned char*>(d_workspace);
    e = hipMemcpyAsync(ws + p->off_tab, p->tables.data(), p->tables.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return device_fail(e, "table upload");
    ps::GreenBufs gb;
    gb.nx = p->nx;
    gb.ny = p->ny;
    gb.nz = p->nz;
    gb.g1 = reinterpret_cast<double*>(ws + p->off_gscr);
    gb.ghat = ws + p->off_ghat;
    for (int a = 0; a < 3; ++a) gb.twf64[a] = ws + p->off_tab + p->tw_f64[a];
    gb.dx = p->dx;
    gb.sy = p->dy / p->dx;
    gb.sz = p->dz / p->dx;
    gb.self_value = self_value(p->dx, p->dy, p->dz, self_coeff);
    const double P3 = (double)axis_pad(p, 0) * axis_pad(p, 1) * axis_pad(p, 2);
    gb.scale = G * p->dx * p->dy * p->dz / P3;
    gb.out_f32 = !is_f64(p->prec);
    gb.plain_layout = is_plain(p->prec);
    gb.stream = st;
    e = ps::green_run(gb);
    if (e != hipSuccess) return device_fail(e, "kernel build launch");
    p->ws = ws;
    ps::SolveRec rec{};
    if (!is_plain(p->prec)) {
        rec = solve_rec(p, nullptr, nullptr);
        e = hipMemcpyAsync(ws + p->off_rec, &rec, sizeof(rec), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return device_fail(e, "solve record upload");
    }
    e = hipStreamSynchronize(st);  // also ends the uploads from host memory
    if (e != hipSuccess) return device_fail(e, "kernel build");
    p->G = G;
    p->self_coeff = self_coeff;
    p->ready = true;
    p->batch_sig.clear();  // a rebuilt plan invalidates any uploaded batch records
    return PS_OK;
}

ps_status ps_solve(ps_plan p, const void* d_rho, void* d_phi, void* stream)
{
    if (ps_status s = check_plan(p)) return s;
    if (!d_rho || !d_phi) return fail(PS_ERR_INVALID, "rho and phi must be non-NULL");
    if ((uintptr_t)d_rho % p->real_bytes || (uintptr_t)d_phi % p->real_bytes)
        return fail(PS_ERR_INVALID, "rho and phi must be aligned to their element size");
    const size_t bytes = cells(p) * p->real_bytes;
    if (overlap(d_rho, bytes, d_phi, bytes)) return fail(PS_ERR_INVALID, "rho and phi overlap");
    if (!p->ready) return fail(PS_ERR_NOT_READY, "call ps_green_build first");
    const hipError_t e = enqueue_solve(p, d_rho, d_phi, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "solve launch");
    return PS_OK;
}

ps_status ps_solve_static(ps_plan p, const void* d_rho, void* d_phi, void* stream)
{
    if (ps_status s = check_plan(p)) return s;
    if (is_plain(p->prec)) return fail(PS_ERR_UNSUPPORTED, "ps_solve_static runs the pruned pipeline only");
    if (!d_rho || !d_phi) return fail(PS_ERR_INVALID, "rho and phi must be non-NULL");
    if ((uintptr_t)d_rho % p->real_bytes || (uintptr_t)d_phi % p->real_bytes)
        return fail(PS_ERR_INVALID, "rho and phi must be aligned to their element size");
    const size_t bytes = cells(p) * p->real_bytes;
    if (overlap(d_rho, bytes, d_phi, bytes)) return fail(PS_ERR_INVALID, "rho and phi overlap");
    // T1/T4, T2 and T3 back to back, each 256-byte aligned
    const size_t o2 = align_up(p->off_t2 - p->off_t1), o3 = o2 + align_up(p->off_t3 - p->off_t2);
    const size_t need = o3 + align_up(p->off_t3 - p->off_t2);
    if (need > ps::STATIC_SCRATCH_BYTES)
        return fail(PS_ERR_UNSUPPORTED, "this plan needs " + std::to_string(need) +
                                            " bytes of scratch; the static scratch holds " +
                                            std::to_string(ps::STATIC_SCRATCH_BYTES));
    if (!p->ready) return fail(PS_ERR_NOT_READY, "call ps_green_build first");
    void* scr = nullptr;
    hipError_t e = ps::static_scratch(&scr);
    if (e != hipSuccess) return device_fail(e, "static scratch address");
    unsigned char* s1 = static_cast<unsigned char*>(scr);
    ps::PrunedBufs b = pruned_bufs(p, d_rho, d_phi, (hipStream_t)stream);
    b.out[0] = s1;
    b.in[1] = s1;
    b.out[1] = s1 + o2;
    b.in[2] = s1 + o2;
    b.out[2] = s1 + o3;
    b.in[3] = s1 + o3;
    b.out[3] = s1;
    b.in[4] = s1;
    e = run_pruned(p->prec, 0, 5, b);
    if (e != hipSuccess) return device_fail(e, "solve launch");
    return PS_OK;
}

ps_status ps_host_stage_bytes(ps_plan p, size_t* bytes)
{
    if (ps_status s = check_plan(p)) return s;
    if (!bytes) return fail(PS_ERR_INVALID, "bytes is NULL");
    *bytes = host_stage_bytes(p);
    return PS_OK;
}

ps_status ps_solve_host(ps_plan p, const void* const* h_rho, void* const* h_phi, int count, void* d_stage,
                        size_t stage_bytes, void* stream)
{
    if (ps_status s = check_plan(p)) return s;
    if (!h_rho || !h_phi) return fail(PS_ERR_INVALID, "rho and phi lists must be non-NULL");
    if (count <= 0) return fail(PS_ERR_INVALID, "count must be positive");
    const size_t bytes = cells(p) * p->real_bytes;
    for (int i = 0; i < count; ++i) {
        if (!h_rho[i] || !h_phi[i]) return fail(PS_ERR_INVALID, "solve " + std::to_string(i) + ": NULL array");
        if (overlap(h_rho[i], bytes, h_phi[i], bytes))
            return fail(PS_ERR_INVALID, "solve " + std::to_string(i) + ": rho and phi overlap");
    }
    // the download of one solve runs while later uploads read their inputs:
    // no output may overlap another solve's input or output
    for (int i = 0; i < count; ++i)
        for (int j = 0; j < count; ++j)
            if (j != i && (overlap(h_phi[i], bytes, h_rho[j], bytes) || overlap(h_phi[i], bytes, h_phi[j], bytes)))
                return fail(PS_ERR_INVALID, "output of solve " + std::to_string(i) + " overlaps an array of solve " +
                                                std::to_string(j));
    if (!d_stage) return fail(PS_ERR_INVALID, "staging memory is NULL");
    if ((uintptr_t)d_stage % ALIGN) return fail(PS_ERR_INVALID, "staging memory must be 256-byte aligned");
    if (stage_bytes < host_stage_bytes(p)) return fail(PS_ERR_INVALID, "staging memory smaller than ps_host_stage_bytes");
    if (!p->ready) return fail(PS_ERR_NOT_READY, "call ps_green_build first");
    hipStream_t st = (hipStream_t)stream;
    bool cap = false;
    hipError_t e;
    if (!capturing(st, cap, e)) return device_fail(e, "hipStreamIsCapturing");
    if (cap) return fail(PS_ERR_CAPTURE, "host-resident solves cannot run under stream capture");
    if (!p->up) {
        if ((e = hipStreamCreateWithFlags(&p->up, hipStreamNonBlocking)) != hipSuccess)
            return device_fail(e, "hipStreamCreateWithFlags");
        if ((e = hipStreamCreateWithFlags(&p->down, hipStreamNonBlocking)) != hipSuccess)
            return device_fail(e, "hipStreamCreateWithFlags");
        for (hipEvent_t& ev : p->hev)
            if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
                return device_fail(e, "hipEventCreateWithFlags");
    }
    // two slots per direction: rho[0], rho[1], phi[0], phi[1]
    unsigned char* stage = static_cast<unsigned char*>(d_stage);
    const size_t slot = align_up(bytes);
    auto d_rho = [&](int s2) { return stage + s2 * slot; };
    auto d_phi = [&](int s2) { return stage + (2 + s2) * slot; };
    hipEvent_t fork = p->hev[0], *up_done = p->hev + 1, *comp_done = p->hev + 3, *down_done = p->hev + 5;
    e = hipEventRecord(fork, st);  // the copies follow earlier work on `stream`
    if (e == hipSuccess) e = hipStreamWaitEvent(p->up, fork, 0);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->down, fork, 0);
    for (int i = 0; i < count && e == hipSuccess; ++i) {
        const int s2 = i & 1;
        // upload i once solve i - 2 has read this input slot
        if (i >= 2) e = hipStreamWaitEvent(p->up, comp_done[s2], 0);
        if (e == hipSuccess) e = hipMemcpyAsync(d_rho(s2), h_rho[i], bytes, hipMemcpyHostToDevice, p->up);
        if (e == hipSuccess) e = hipEventRecord(up_done[s2], p->up);
        // solve i once its input is in and download i - 2 has read this output slot
        if (e == hipSuccess) e = hipStreamWaitEvent(st, up_done[s2], 0);
        if (e == hipSuccess && i >= 2) e = hipStreamWaitEvent(st, down_done[s2], 0);
        if (e == hipSuccess) e = enqueue_solve(p, d_rho(s2), d_phi(s2), st);
        if (e == hipSuccess) e = hipEventRecord(comp_done[s2], st);
        // download i once solve i is done
        if (e == hipSuccess) e = hipStreamWaitEvent(p->down, comp_done[s2], 0);
        if (e == hipSuccess) e = hipMemcpyAsync(h_phi[i], d_phi(s2), bytes, hipMemcpyDeviceToHost, p->down);
        if (e == hipSuccess) e = hipEventRecord(down_done[s2], p->down);
    }
    // `stream` resumes after the last downloads
    for (int s2 = 0; s2 < 2 && s2 < count && e == hipSuccess; ++s2) e = hipStreamWaitEvent(st, down_done[s2], 0);
    if (e != hipSuccess) return device_fail(e, "host-resident solves");
    return PS_OK;
}

ps_status ps_stream_copy(const void* d_src, void* d_dst, size_t bytes, void* stream)
{
    if (!d_src || !d_dst) return fail(PS_ERR_INVALID, "src and dst must be non-NULL");
    if ((uintptr_t)d_src % 16 || (uintptr_t)d_dst % 16 || bytes % 16)
        return fail(PS_ERR_INVALID, "src, dst and bytes must be multiples of 16");
    if (overlap(d_src, bytes, d_dst, bytes)) return fail(PS_ERR_INVALID, "src and dst overlap");
    const hipError_t e = ps::stream_copy(d_src, d_dst, bytes, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "copy launch");
    return PS_OK;
}

ps_status ps_debug_pass(ps_plan p, int pass, const void* d_in, void* d_out, void* stream)
{
    if (ps_status s = check_plan(p)) return s;
    if (is_plain(p->prec)) return fail(PS_ERR_UNSUPPORTED, "debug passes exist for the pruned pipeline only");
    if (pass < 0 || pass > 4) return fail(PS_ERR_INVALID, "pass must be 0..4");
    if (!d_in || !d_out) return fail(PS_ERR_INVALID, "in and out must be non-NULL");
    if (d_in == d_out) return fail(PS_ERR_INVALID, "passes do not run in place");
    if (!p->ready) return fail(PS_ERR_NOT_READY, "call ps_green_build first");
    hipStream_t st = (hipStream_t)stream;
    ps::PrunedBufs b = pruned_bufs(p, nullptr, nullptr, st);
    b.in[pass] = d_in;
    b.out[pass] = d_out;
    hipError_t e = run_pruned(p->prec, pass, pass + 1, b);
    if (e != hipSuccess) return device_fail(e, "pass launch");
    return PS_OK;
}

ps_status ps_plan_set_variant(ps_plan p, int pass, int variant)
{
    if (ps_status s = check_plan(p)) return s;
    if (is_plain(p->prec)) return fail(PS_ERR_UNSUPPORTED, "plain plans have no variants");
    if (pass == 5) {
        if (p->prec != PS_F32_SPLIT) return fail(PS_ERR_UNSUPPORTED, "product terms apply to PS_F32_SPLIT plans");
        if (variant != 3 && variant != 6) return fail(PS_ERR_INVALID, "split product terms must be 3 or 6");
        p->var.mterms = variant;
        return PS_OK;
    }
    if (pass == 6) {
        if (variant != 0 && variant != 1) return fail(PS_ERR_INVALID, "z tile must be 0 (full) or 1 (half)");
        p->var.ztile = variant;
        return PS_OK;
    }
    if (pass < 0 || pass > 4) return fail(PS_ERR_INVALID, "pass must be 0..6");
    if (variant < 0 || variant >= num_variants(pass)) return fail(PS_ERR_INVALID, "variant out of range");
    if (variant_needs_family1(pass, variant) && !family1_available(p, pass))
        return fail(PS_ERR_UNSUPPORTED, "this plan has no radix-32 plan family");
    if (!variant_ok(p, pass, variant))
        return fail(PS_ERR_UNSUPPORTED, (pass == 0 || pass == 4)
                                            ? "this x tile does not fit the LDS, or boxes (16 rows per x tile only)"
                                            : "boxes run the one-tile-per-workgroup kernels (no persistent variants)");
    *variant_slot(p->var, pass) = variant;
    return PS_OK;
}

ps_status ps_plan_set_spacing(ps_plan p, double dy, double dz)
{
    if (ps_status s = check_plan(p)) return s;
    if (!(dy > 0.0) || !(dz > 0.0) || !std::isfinite(dy) || !std::isfinite(dz))
        return fail(PS_ERR_INVALID, "dy and dz must be positive and finite");
    p->dy = dy;
    p->dz = dz;
    p->ready = false;  // the kernel spectrum depends on the spacings
    p->batch_sig.clear();
    return PS_OK;
}

ps_status ps_autotune(ps_plan p, void* stream, const char* cache_path)
{
    if (ps_status s = check_plan(p)) return s;
    if (is_plain(p->prec)) return fail(PS_ERR_UNSUPPORTED, "plain plans have no variants");
    if (!p->ready) return fail(PS_ERR_NOT_READY, "call ps_green_build first");
    hipStream_t st = (hipStream_t)stream;
    bool cap = false;
    hipError_t e;
    if (!capturing(st, cap, e)) return device_fail(e, "hipStreamIsCapturing");
    if (cap) return fail(PS_ERR_CAPTURE, "ps_autotune cannot run under stream capture");
    // rho and phi stand-ins: the start of T2, which passes 0 and 4 do not touch
    ps::PrunedBufs b = pruned_bufs(p, p->ws + p->off_t2, p->ws + p->off_t2, st);
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return device_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        hipEventDestroy(e0);
        return device_fail(e, "hipEventCreate");
    }
    ps_status rc = PS_OK;
    ps::PrunedVariant best = p->var;
    for (int pass = 0; pass < 5 && rc == PS_OK; ++pass) {
        float best_ms = 1e30f;
        // the z pass: every form at both tile widths
        for (int vt = 0; vt < num_variants(pass) * (pass == 2 ? 2 : 1); ++vt) {
            const int v = vt % num_variants(pass);
            if (!variant_ok(p, pass, v)) continue;
            *variant_slot(b.var, pass) = v;
            if (pass == 2) b.var.ztile = vt / num_variants(pass);
            const int reps = 5;
            float ms = 0.f;
            for (int r = 0; r <= reps && rc == PS_OK; ++r) {
                hipEventRecord(e0, st);
                e = run_pruned(p->prec, pass, pass + 1, b);
                hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float t = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
                if (e != hipSuccess) rc = device_fail(e, "autotune");
                if (r > 0) ms += t;  // the first run is a warm-up
            }
            if (rc == PS_OK && ms < best_ms) {
                best_ms = ms;
                *variant_slot(best, pass) = v;
                if (pass == 2) best.ztile = b.var.ztile;
            }
        }
        *variant_slot(b.var, pass) = *variant_slot(best, pass);
        if (pass == 2) b.var.ztile = best.ztile;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc != PS_OK) return rc;
    p->var = best;
    if (cache_path && !p->box && !write_tuning(cache_path, p->P, p->prec, best))
        return fail(PS_ERR_INVALID, std::string("cannot write tuning cache ") + cache_path);
    return PS_OK;
}

ps_status ps_solve_batched(const ps_plan* plans, int count, const void* const* d_rho, void* const* d_phi,
                           void* stream)
{
    if (!plans || !d_rho || !d_phi) return fail(PS_ERR_INVALID, "plans, rho and phi lists must be non-NULL");
    if (count <= 0) return fail(PS_ERR_INVALID, "count must be positive");
    if (count > MAX_BATCH) return fail(PS_ERR_UNSUPPORTED, "at most " + std::to_string(MAX_BATCH) + " solves per batch");
    for (int i = 0; i < count; ++i)
        if (!plans[i]) return fail(PS_ERR_INVALID, "plan " + std::to_string(i) + " is NULL");
    const ps_precision prec = plans[0]->prec;
    if (is_plain(prec)) return fail(PS_ERR_UNSUPPORTED, "batched solves use the pruned pipeline");
    for (int i = 0; i < count; ++i) {
        const ps_plan p = plans[i];
        const std::string who = "solve " + std::to_string(i);
        if (p->prec != prec) return fail(PS_ERR_INVALID, who + ": all plans of a batch need the same precision");
        if (!d_rho[i] || !d_phi[i]) return fail(PS_ERR_INVALID, who + ": rho and phi must be non-NULL");
        if ((uintptr_t)d_rho[i] % p->real_bytes || (uintptr_t)d_phi[i] % p->real_bytes)
            return fail(PS_ERR_INVALID, who + ": rho and phi must be aligned to their element size");
        for (int j = 0; j < i; ++j)
            if (plans[j] == p) return fail(PS_ERR_INVALID, who + ": a plan may appear once per batch");
    }
    for (int i = 0; i < count; ++i) {
        const size_t bi = cells(plans[i]) * plans[i]->real_bytes;
        if (overlap(d_rho[i], bi, d_phi[i], bi)) return fail(PS_ERR_INVALID, "rho and phi overlap");
        for (int j = 0; j < count; ++j) {
            if (j == i) continue;
            const size_t bj = cells(plans[j]) * plans[j]->real_bytes;
            if (overlap(d_phi[i], bi, d_phi[j], bj) || overlap(d_phi[i], bi, d_rho[j], bj))
                return fail(PS_ERR_INVALID, "output of solve " + std::to_string(i) + " overlaps another array");
        }
    }
    for (int i = 0; i < count; ++i)
        if (!plans[i]->ready) return fail(PS_ERR_NOT_READY, "solve " + std::to_string(i) + ": call ps_green_build first");
    hipStream_t st = (hipStream_t)stream;
    ps_plan head = plans[0];
    // Members sorted by size (largest first) and shape, then by kernel
    // variants, so that per pass every run of equal-shape members with the
    // same kernel is one launch over their adjacent records.
    auto vkey = [&](int i) {
        const ps::PrunedVariant& v = plans[i]->var;
        return std::array<int, 11>{-plans[i]->nx * plans[i]->ny * plans[i]->nz, -plans[i]->nz, -plans[i]->ny,
                                  -plans[i]->nx, v.x_fam, v.y_fam, v.zmode, v.yi_fam, v.xc_fam, v.mterms, v.ztile};
    };
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return vkey(a) < vkey(b); });
    std::vector<uintptr_t> sig;
    sig.push_back((uintptr_t)count);
    for (int k = 0; k < count; ++k) {
        const int i = order[k];
        sig.push_back((uintptr_t)plans[i]);
        sig.push_back((uintptr_t)d_rho[i]);
        sig.push_back((uintptr_t)d_phi[i]);
        sig.push_back((uintptr_t)plans[i]->ws);
        for (int x : vkey(i)) sig.push_back((uintptr_t)(intptr_t)x);
    }
    auto* dlist = reinterpret_cast<ps::SolveRec*>(head->ws + head->off_batch);
    // per pass, runs [k0, k1) of equal shape and equal kernel variant
    std::vector<std::pair<int, int>> groups[5];
    size_t most = 1;
    for (int pass = 0; pass < 5; ++pass) {
        for (int k0 = 0; k0 < count;) {
            ps::PrunedVariant v0 = plans[order[k0]]->var;
            int k1 = k0 + 1;
            while (k1 < count) {
                ps::PrunedVariant v1 = plans[order[k1]]->var;
                const ps_plan a = plans[order[k0]], c = plans[order[k1]];
                if (c->nx != a->nx || c->ny != a->ny || c->nz != a->nz ||
                    *variant_slot(v1, pass) != *variant_slot(v0, pass) || v1.mterms != v0.mterms ||
                    (pass == 2 && v1.ztile != v0.ztile))
                    break;
                ++k1;
            }
            groups[pass].emplace_back(k0, k1);
            k0 = k1;
        }
        most = std::max(most, groups[pass].size());
    }
    if (sig != head->batch_sig) {
        bool cap = false;
        hipError_t e;
        if (!capturing(st, cap, e)) return device_fail(e, "hipStreamIsCapturing");
        if (cap) return fail(PS_ERR_CAPTURE, "the first call with a new batch uploads its records; not under capture");
        std::vector<ps::SolveRec> recs(count);
        for (int k = 0; k < count; ++k) recs[k] = solve_rec(plans[order[k]], d_rho[order[k]], d_phi[order[k]]);
        e = hipMemcpyAsync(dlist, recs.data(), recs.size() * sizeof(ps::SolveRec), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host array is released on return
        if (e != hipSuccess) return device_fail(e, "batch record upload");
        // groups of one pass run side by side: one extra stream per group beyond the first
        if (most > 1 && !head->fork) {
            if ((e = hipEventCreateWithFlags(&head->fork, hipEventDisableTiming)) != hipSuccess)
                return device_fail(e, "hipEventCreateWithFlags");
        }
        while (head->aux.size() + 1 < most) {
            hipStream_t s2 = nullptr;
            hipEvent_t e2 = nullptr;
            if ((e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking)) != hipSuccess)
                return device_fail(e, "hipStreamCreateWithFlags");
            head->aux.push_back(s2);
            if ((e = hipEventCreateWithFlags(&e2, hipEventDisableTiming)) != hipSuccess)
                return device_fail(e, "hipEventCreateWithFlags");
            head->join.push_back(e2);
        }
        head->batch_sig = sig;
    }
    for (int pass = 0; pass < 5; ++pass) {
        const auto& gr = groups[pass];
        hipError_t e = hipSuccess;
        if (gr.size() > 1) e = hipEventRecord(head->fork, st);
        for (size_t g = 0; g < gr.size() && e == hipSuccess; ++g) {
            hipStream_t sg = g == 0 ? st : head->aux[g - 1];
            if (g > 0) e = hipStreamWaitEvent(sg, head->fork, 0);
            if (e != hipSuccess) break;
            const ps_plan p0 = plans[order[gr[g].first]];
            ps::PrunedBufs b = pruned_bufs(p0, nullptr, nullptr, sg);
            b.list = dlist + gr[g].first;
            b.count = gr[g].second - gr[g].first;
            e = run_pruned(prec, pass, pass + 1, b);
            if (e == hipSuccess && g > 0) e = hipEventRecord(head->join[g - 1], sg);
        }
        for (size_t g = 1; g < gr.size() && e == hipSuccess; ++g) e = hipStreamWaitEvent(st, head->join[g - 1], 0);
        if (e != hipSuccess) return device_fail(e, "batched launch");
    }
    return PS_OK;
}

}  // extern "C"
