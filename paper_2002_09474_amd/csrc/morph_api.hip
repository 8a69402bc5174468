// Host side of the HIP morphology library: argument checks, per-pass method
// choice (direct below a window threshold, van Herk/Gil-Werman above it, the
// paper's hybrid of §5.3), tile planning, launches, open/close compositions, the
// batched persistent launch and the tuning table.
#include "../../include/morph.h"
#include "morph_internal.h"

#include <algorithm>
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace morph;

namespace {

thread_local int g_last_hip_error = 0;

int hip_fail(hipError_t e)
{
    g_last_hip_error = (int)e;
    return MORPH_EHIP;
}

// ---------------- tuning table ----------------
// Tile shape for windows up to wmax: the tile's input row spans tq quads of 4
// pixels (so the vertical pass has tq work units per band of rows) and the tile
// has tb output rows.
struct TileRule {
    int wmax; // applies when max(wx, wy) <= wmax
    int tq, tb;
};

struct DtypeTuning {
    int t_x, t_y; // direct when w <= t (per pass)
    std::vector<TileRule> tiles;
    int wave_rows;   // output rows of a wave unit (both passes direct), multiple of kWaveRows
    int stream_rows;      // output rows of a streaming-kernel unit (LDS-ring form)
    int stream_rows_runs; // the same for the run-total form (wy > kStreamRingMaxWy)
    int wide_rows;        // output rows of a wide-row unit (wy 1, wx > kStreamMaxWx)
    int fuse;             // batches: wave and streaming groups in one dispatch (0 / 1)
    // the unit heights above for images of a batch, whose many units fill the GPU
    // whatever their height, so that longer units (less vertical warm-up) pay
    int batch_wave_rows, batch_stream_rows, batch_stream_rows_runs;
    int fit_units; // single images: shorten units until the launch fills the GPU (0 / 1)
    // the thresholds for the images of a batch, measured on a batch: there a pass that
    // leaves the fused dispatch (the wave kernel's tall form) can cost more than it
    // saves on its own images
    int batch_t_x, batch_t_y;
    // single images' openings and closings in one pass where it applies (0 / 1), the
    // output rows of its units (multiples of kWaveRows; vertical windows up to kDirectMax,
    // then the tall ones), and the largest horizontal window its passes take direct
    // (doubling above)
    int oc_one_pass, oc_rows, oc_t_x, oc_rows_tall;
    // output rows of a unit of the wave kernel's tall form (vertical windows past
    // kDirectMax; single images and batches), a multiple of kWaveRows
    int wave_rows_tall;
    // single images' automatic large horizontal windows: 0 = doubling across the lanes,
    // 1 = the paper's vHGW across the lanes (where a kernel has that form)
    int h_vhgw;
    // single images on aligned rows with vertical vHGW in run totals and wy >= coop_min_wy
    // (0: never) take the streaming kernel's cooperative form, units of coop_rows rows
    // shared by coop_waves waves (4, 8 or 16); the same three for the images of a batch
    // (whose cooperative units run as a dispatch of their own)
    int coop_min_wy, coop_rows, coop_waves;
    int batch_coop_min_wy, batch_coop_rows, batch_coop_waves;
};

std::mutex g_tuning_mu;
// The autotuner's table for gfx950 (its sweeps are kept in tuning_gfx950.json next to
// the Python package): direct passes up to 9 along x (16 for uint16) and 31 along y on
// single images, 9 and 9 for the images of a batch; unit heights and tile shapes.
const DtypeTuning k_builtin_tuning[2] = {
    {12, 31, {{9, 32, 64}, {16, 64, 32}, {32, 64, 32}, {64, 64, 32}, {1 << 30, 48, 32}}, 8, 96, 32, 4,
     1, 16, 48, 64, 1, 9, 9, 1, 16, 9, 48, 8, 0, 33, 96, 8, 0, 96, 8},
    {16, 31, {{9, 32, 64}, {16, 64, 32}, {32, 64, 32}, {64, 64, 32}, {1 << 30, 48, 32}}, 8, 64, 24, 4,
     1, 16, 64, 64, 1, 9, 9, 1, 8, 9, 48, 16, 0, 33, 96, 8, 0, 96, 8},
};
DtypeTuning g_tuning[2] = {k_builtin_tuning[0], k_builtin_tuning[1]};

DtypeTuning tuning_for(int dtype)
{
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    return g_tuning[dtype];
}

// Minimal JSON reader for the tuning file (objects, arrays, numbers, strings).
struct JVal {
    enum Kind { NUL, NUM, STR, ARR, OBJ } k = NUL;
    double num = 0;
    std::string str;
    std::vector<JVal> arr;
    std::map<std::string, JVal> obj;
};

struct JParser {
    const char *p, *e;
    bool ok = true;
    void ws()
    {
        while (p < e && std::isspace((unsigned char)*p)) p++;
    }
    bool parse(JVal &v)
    {
        ws();
        if (p >= e) return false;
        if (*p == '{') {
            v.k = JVal::OBJ;
            p++;
            ws();
            if (p < e && *p == '}') { p++; return true; }
            for (;;) {
                JVal key;
                ws();
                if (!parse(key) || key.k != JVal::STR) return false;
                ws();
                if (p >= e || *p != ':') return false;
                p++;
                JVal val;
                if (!parse(val)) return false;
                v.obj[key.str] = val;
                ws();
                if (p < e && *p == ',') { p++; continue; }
                if (p < e && *p == '}') { p++; return true; }
                return false;
            }
        }
        if (*p == '[') {
            v.k = JVal::ARR;
            p++;
            ws();
            if (p < e && *p == ']') { p++; return true; }
            for (;;) {
                JVal el;
                if (!parse(el)) return false;
                v.arr.push_back(el);
                ws();
                if (p < e && *p == ',') { p++; continue; }
                if (p < e && *p == ']') { p++; return true; }
                return false;
            }
        }
        if (*p == '"') {
            v.k = JVal::STR;
            p++;
            while (p < e && *p != '"') {
                if (*p == '\\' && p + 1 < e) p++;
                v.str.push_back(*p++);
            }
            if (p >= e) return false;
            p++;
            return true;
        }
        if (!std::strncmp(p, "null", 4)) { p += 4; v.k = JVal::NUL; return true; }
        if (!std::strncmp(p, "true", 4)) { p += 4; v.k = JVal::NUM; v.num = 1; return true; }
        if (!std::strncmp(p, "false", 5)) { p += 5; v.k = JVal::NUM; v.num = 0; return true; }
        char *end = nullptr;
        v.num = std::strtod(p, &end);
        if (end == p) return false;
        v.k = JVal::NUM;
        p = end;
        return true;
    }
};

bool read_dtype_tuning(const JVal &o, DtypeTuning &t)
{
    if (o.k != JVal::OBJ) return false;
    auto it = o.obj.find("t_x");
    if (it != o.obj.end() && it->second.k == JVal::NUM) t.t_x = (int)it->second.num;
    it = o.obj.find("t_y");
    if (it != o.obj.end() && it->second.k == JVal::NUM) t.t_y = (int)it->second.num;
    it = o.obj.find("batch_t_x");
    if (it != o.obj.end() && it->second.k == JVal::NUM) t.batch_t_x = (int)it->second.num;
    it = o.obj.find("batch_t_y");
    if (it != o.obj.end() && it->second.k == JVal::NUM) t.batch_t_y = (int)it->second.num;
    const struct {
        const char *key;
        int DtypeTuning::*field;
    } chunk_keys[] = {{"wave_rows", &DtypeTuning::wave_rows},
                      {"batch_wave_rows", &DtypeTuning::batch_wave_rows},
                      {"oc_rows", &DtypeTuning::oc_rows},
                      {"oc_rows_tall", &DtypeTuning::oc_rows_tall},
                      {"wave_rows_tall", &DtypeTuning::wave_rows_tall}};
    for (const auto &ck : chunk_keys) { // (whole chunks of kWaveRows rows)
        it = o.obj.find(ck.key);
        if (it == o.obj.end()) continue;
        if (it->second.k != JVal::NUM) return false;
        const int r = (int)it->second.num;
        if (r < kWaveRows || r > 8 * kWaveRows || r % kWaveRows) return false;
        t.*ck.field = r;
    }
    const struct {
        const char *min_wy, *rows, *waves;
        int DtypeTuning::*f_min_wy, DtypeTuning::*f_rows, DtypeTuning::*f_waves;
    } coop_keys[] = {{"coop_min_wy", "coop_rows", "coop_waves", &DtypeTuning::coop_min_wy,
                      &DtypeTuning::coop_rows, &DtypeTuning::coop_waves},
                     {"batch_coop_min_wy", "batch_coop_rows", "batch_coop_waves",
                      &DtypeTuning::batch_coop_min_wy, &DtypeTuning::batch_coop_rows,
                      &DtypeTuning::batch_coop_waves}};
    for (const auto &ck : coop_keys) {
        it = o.obj.find(ck.min_wy);
        if (it != o.obj.end()) {
            if (it->second.k != JVal::NUM) return false;
            const int r = (int)it->second.num;
            if (r < 0) return false;
            t.*ck.f_min_wy = r;
        }
        it = o.obj.find(ck.rows);
        if (it != o.obj.end()) {
            if (it->second.k != JVal::NUM) return false;
            const int r = (int)it->second.num;
            if (r < 8 || r > 1024 || r % 8) return false;
            t.*ck.f_rows = r;
        }
        it = o.obj.find(ck.waves);
        if (it != o.obj.end()) {
            if (it->second.k != JVal::NUM) return false;
            const int r = (int)it->second.num;
            if (r != 4 && r != 8 && r != 16) return false;
            t.*ck.f_waves = r;
        }
    }
    it = o.obj.find("oc_t_x");
    if (it != o.obj.end()) {
        if (it->second.k != JVal::NUM) return false;
        const int r = (int)it->second.num;
        if (r < 1) return false;
        t.oc_t_x = std::min(r, kDirectMax);
    }
    const struct {
        const char *key;
        int DtypeTuning::*field;
    } flag_keys[] = {{"oc_one_pass", &DtypeTuning::oc_one_pass},
                     {"h_vhgw", &DtypeTuning::h_vhgw},
                     {"fit_units", &DtypeTuning::fit_units},
                     {"fuse", &DtypeTuning::fuse}};
    for (const auto &fk : flag_keys) { // (0 or 1)
        it = o.obj.find(fk.key);
        if (it == o.obj.end()) continue;
        if (it->second.k != JVal::NUM) return false;
        const int r = (int)it->second.num;
        if (r != 0 && r != 1) return false;
        t.*fk.field = r;
    }
    it = o.obj.find("wide_rows");
    if (it != o.obj.end()) {
        if (it->second.k != JVal::NUM) return false;
        const int r = (int)it->second.num;
        if (r < 1 || r > 4096) return false;
        t.wide_rows = r;
    }
    const struct {
        const char *key;
        int DtypeTuning::*field;
    } rows_keys[] = {{"stream_rows", &DtypeTuning::stream_rows},
                     {"stream_rows_runs", &DtypeTuning::stream_rows_runs},
                     {"batch_stream_rows", &DtypeTuning::batch_stream_rows},
                     {"batch_stream_rows_runs", &DtypeTuning::batch_stream_rows_runs}};
    for (const auto &rk : rows_keys) {
        it = o.obj.find(rk.key);
        if (it == o.obj.end()) continue;
        if (it->second.k != JVal::NUM) return false;
        const int r = (int)it->second.num;
        if (r < 1 || r > 4096) return false;
        t.*rk.field = r;
    }
    it = o.obj.find("tiles");
    if (it != o.obj.end()) {
        if (it->second.k != JVal::ARR) return false;
        std::vector<TileRule> rules;
        for (const JVal &r : it->second.arr) {
            if (r.k != JVal::OBJ) return false;
            auto w = r.obj.find("wmax"), a = r.obj.find("tq"), b = r.obj.find("tb");
            if (w == r.obj.end() || a == r.obj.end() || b == r.obj.end()) return false;
            TileRule tr{(int)w->second.num, (int)a->second.num, (int)b->second.num};
            if (tr.tq < 2 || tr.tq > 4096 || tr.tb < 2 || tr.tb % 2) return false;
            rules.push_back(tr);
        }
        std::sort(rules.begin(), rules.end(),
                  [](const TileRule &x, const TileRule &y) { return x.wmax < y.wmax; });
        if (!rules.empty()) {
            rules.back().wmax = std::max(rules.back().wmax, 1 << 30);
            t.tiles = rules;
        }
    }
    return t.t_x >= 1 && t.t_y >= 1 && t.batch_t_x >= 1 && t.batch_t_y >= 1;
}

// ---------------- planning ----------------
size_t elem_bytes(int dtype) { return dtype == MORPH_U16 ? 2 : 1; }

int check_image(int dtype, const void *src, const void *dst, int H, int W, size_t pitch, int wx,
                int wy, int ax, int ay, int border)
{
    if (dtype != MORPH_U8 && dtype != MORPH_U16) return MORPH_EUNSUPPORTED;
    if (border != MORPH_BORDER_NEUTRAL) return MORPH_EUNSUPPORTED;
    if (H < 0 || W < 0) return MORPH_EINVAL;
    if (wx < 1 || wy < 1) return MORPH_EINVAL;
    if (ax < -1 || ax >= wx || ay < -1 || ay >= wy) return MORPH_EINVAL;
    if (H == 0 || W == 0) return MORPH_OK;
    const size_t es = elem_bytes(dtype);
    if (!src || !dst) return MORPH_EINVAL;
    if (pitch < (size_t)W * es || pitch % es) return MORPH_EINVAL;
    if (pitch > (size_t)1 << 40) return MORPH_EINVAL;
    if (es == 2 && (((uintptr_t)src | (uintptr_t)dst) & 1)) return MORPH_EINVAL;
    return MORPH_OK;
}

bool ranges_overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

size_t image_span(int H, int W, size_t pitch, int dtype)
{
    return (size_t)(H - 1) * pitch + (size_t)W * elem_bytes(dtype);
}

int default_anchor(int w) { return w - 1 - w / 2; }

// Single images: a wave or streaming unit's rows go one chunk after another, so an
// image with fewer units than the GPU holds waves finishes in about one unit's time,
// which grows with its height.  Units are shortened (in steps of 8 rows, to no fewer
// than 8) until the launch has about kUnitTarget of them: 8 waves per CU of a 256-CU
// MI355X.  Batches fill the GPU with many images and keep the tuned heights.
constexpr int kUnitTarget = 2048;

// Output quads a strip of the wave or streaming kernel stores: no more than sq (those
// whose input lies in the wave's 64 quads), as few strips as that allows, and the
// strips as even as possible (a 1920-pixel row: 8 strips of 60 quads, none partial).
static int strip_quads(int W, int sq)
{
    const int nq = (W + 3) / 4;
    const int n = (nq + sq - 1) / sq;
    return (nq + n - 1) / n;
}

static int fit_rows(int tuned, int H, int strips)
{
    const int64_t need = ((int64_t)H * strips + kUnitTarget - 1) / kUnitTarget; // rows a unit
    const int tb = (int)std::min<int64_t>(tuned, (need + 7) / 8 * 8);
    return std::max(std::min(tuned, 8), tb);
}

// Fill a TileJob for one erosion/dilation.  Windows are clipped to the image: with
// anchor a and right extent r = w - 1 - a, only min(a, W-1) columns to the left and
// min(r, W-1) to the right can ever be inside the image.
int plan_job(int op, int dtype, const void *src, void *dst, int H, int W, size_t pitch,
             size_t dpitch, int wx, int wy, int ax, int ay, const morph_plan *plan, TileJob &j,
             bool batch = false)
{
    if (ax < 0) ax = default_anchor(wx);
    if (ay < 0) ay = default_anchor(wy);
    const int axe = std::min(ax, W - 1), rxe = std::min(wx - 1 - ax, W - 1);
    const int aye = std::min(ay, H - 1), rye = std::min(wy - 1 - ay, H - 1);
    j.src = (const uint8_t *)src;
    j.dst = (uint8_t *)dst;
    j.H = H;
    j.W = W;
    j.pitch = (int64_t)pitch;
    j.dpitch = (int64_t)dpitch;
    j.wx = axe + rxe + 1;
    j.wy = aye + rye + 1;
    j.ax = axe;
    j.ay = aye;
    j.op = op;
    j.dtype = dtype;
    j.keep = 0;

    const DtypeTuning tu = tuning_for(dtype);
    const int mx = plan ? plan->method_x : MORPH_METHOD_AUTO;
    const int my = plan ? plan->method_y : MORPH_METHOD_AUTO;
    const bool user_tile = plan && (plan->tile_w > 0 || plan->tile_h > 0);
    if (mx < 0 || mx > 3 || my < 0 || my > 2) return MORPH_EINVAL;
    if (mx == MORPH_METHOD_DOUBLING && user_tile) return MORPH_EINVAL;
    const bool auto_both = mx == MORPH_METHOD_AUTO && my == MORPH_METHOD_AUTO;
    const bool stream_fits = j.wx <= kStreamMaxWx && j.wy <= kStreamMaxWy;
    // rows with a window too wide for the other kernels' strips (vertical window 1)
    const bool rows_fit = j.wy == 1 && j.wx > kStreamMaxWx && j.wx <= kRowsMaxWx;
    if (mx == MORPH_METHOD_DOUBLING && !stream_fits && !rows_fit) return MORPH_EUNSUPPORTED;
    // horizontal pass
    if (j.wx == 1) j.hm = PASS_NONE;
    else if (mx == MORPH_METHOD_DIRECT) j.hm = PASS_DIRECT;
    else if (mx == MORPH_METHOD_VHGW) j.hm = PASS_VHGW;
    else if (mx == MORPH_METHOD_DOUBLING) j.hm = PASS_DOUBLING;
    else j.hm = (j.wx <= std::min(batch ? tu.batch_t_x : tu.t_x, kDirectMaxX)) ? PASS_DIRECT
                                                                                 : PASS_VHGW;
    // vertical pass (a window of 1 is the direct pass's plain load)
    if (j.wy == 1) j.vm = PASS_DIRECT;
    else if (my == MORPH_METHOD_DIRECT) j.vm = PASS_DIRECT;
    else if (my == MORPH_METHOD_VHGW) j.vm = PASS_VHGW;
    else j.vm = (j.wy <= std::min(batch ? tu.batch_t_y : tu.t_y, kDirectMaxTall)) ? PASS_DIRECT
                                                                                  : PASS_VHGW;
    // (direct windows past the compiled ones run on the tile kernel's tap loops)
    j.vcode = (j.vm == PASS_DIRECT) ? j.wy : 0;
    j.hcode = (j.hm == PASS_NONE) ? 1 : (j.hm == PASS_DIRECT ? j.wx : 0);
    j.SA = j.SB = 0;
    j.vrun = j.vtt = 0;
    j.coop = 0;

    // wide windows along rows: the wide-row kernel (horizontal doubling, 16 pixels a
    // lane), unless a tile or the vHGW passes are asked for
    if (rows_fit && !user_tile && (mx == MORPH_METHOD_AUTO || mx == MORPH_METHOD_DOUBLING) &&
        my != MORPH_METHOD_VHGW) {
        j.kind = KIND_ROWS;
        j.hm = PASS_DOUBLING;
        j.hcode = 0;
        j.TW = 16 * rows_lanes(j.wx);
        j.TB = std::min(tu.wide_rows, H);
        j.tiles_x = (W + j.TW - 1) / j.TW;
        j.tiles_y = (H + j.TB - 1) / j.TB;
        if ((int64_t)j.tiles_x * j.tiles_y > INT32_MAX - 4) return MORPH_EUNSUPPORTED;
        return MORPH_OK;
    }

    // vertical pass direct and no tile asked for: the register-only wave kernel, with
    // the horizontal pass direct or (wider windows, automatic or asked for) doubling
    // A horizontal vHGW asked for (single images, no tile, wx <= kStreamMaxWx) runs
    // across the lanes of the wave or streaming kernel (their XV forms); automatic
    // large horizontal windows take doubling, or that vHGW where the tuning table says
    // so (h_vhgw; the tall wave form has no XV form and keeps doubling).
    j.kind = KIND_TILE;
    const bool lane_vhgw = j.hm == PASS_VHGW && !user_tile && !batch && j.wx <= kStreamMaxWx &&
                           (mx == MORPH_METHOD_VHGW || (mx == MORPH_METHOD_AUTO && tu.h_vhgw));
    const bool h_wave = (j.hm == PASS_DIRECT && j.wx <= kDirectMaxX) || j.hm == PASS_NONE ||
                        j.hm == PASS_DOUBLING ||
                        (j.hm == PASS_VHGW && mx == MORPH_METHOD_AUTO && j.wx <= kStreamMaxWx) ||
                        (lane_vhgw && j.wy <= kDirectMax);
    if (j.vm == PASS_DIRECT && j.wy <= kDirectMaxTall && h_wave && !user_tile &&
        (my != MORPH_METHOD_VHGW)) {
        j.kind = KIND_WAVE;
        if (j.hm == PASS_VHGW && !(lane_vhgw && j.wy <= kDirectMax)) j.hm = PASS_DOUBLING;
        j.hcode = (j.hm == PASS_NONE) ? 1 : (j.hm == PASS_DIRECT ? j.wx : 0);
        // (a strip stores at most the quads whose input lies in its 64 quads,
        // stream_quads(wx) of them, whatever the horizontal pass)
        j.TW = 4 * strip_quads(W, stream_quads(j.wx));
        // (the tall form, a kernel of its own with fewer waves per SIMD, has a height
        // of its own)
        const int rows = j.wy > kDirectMax ? tu.wave_rows_tall
                                           : (batch ? tu.batch_wave_rows : tu.wave_rows);
        j.TB = std::min(rows, (H + kWaveRows - 1) / kWaveRows * kWaveRows);
        j.tiles_x = (W + j.TW - 1) / j.TW;
        if (!batch && tu.fit_units) j.TB = fit_rows(j.TB, H, j.tiles_x);
        j.tiles_y = (H + j.TB - 1) / j.TB;
        if ((int64_t)j.tiles_x * j.tiles_y > INT32_MAX - 4) return MORPH_EUNSUPPORTED;
        return MORPH_OK;
    }
    // doubling asked for, or everything automatic and the windows fit: the streaming
    // kernel (its vertical pass is vHGW through the LDS ring whatever wy is)
    if (j.hm == PASS_DOUBLING || (auto_both && !user_tile && stream_fits) ||
        (lane_vhgw && my != MORPH_METHOD_DIRECT && j.wy <= kStreamMaxWy)) {
        j.kind = KIND_STREAM;
        // (its direct horizontal pass takes windows up to kDirectMax)
        if ((j.hm == PASS_VHGW && !lane_vhgw) || (j.hm == PASS_DIRECT && j.wx > kDirectMax))
            j.hm = PASS_DOUBLING;
        j.vm = PASS_VHGW;
        j.vcode = 0;
        j.hcode = (j.hm == PASS_NONE) ? 1 : (j.hm == PASS_DIRECT ? j.wx : 0);
        j.TW = 4 * strip_quads(W, stream_quads(j.wx));
        j.tiles_x = (W + j.TW - 1) / j.TW;
        // (by measurement: single images, 48 rows for the LDS-ring form and 32 for
        // the run-total form, which give a 4096x4096 image units enough to fill the
        // GPU; in a batch, whose units fill it anyway, 48 for both, which spends less
        // on each unit's vertical warm-up)
        j.TB = std::min(stream_two_level(j.wy) ? (batch ? tu.batch_stream_rows_runs : tu.stream_rows_runs)
                                               : (batch ? tu.batch_stream_rows : tu.stream_rows),
                        H);
        if (!batch && tu.fit_units) j.TB = fit_rows(j.TB, H, j.tiles_x);
        // tall vertical windows on aligned rows: the cooperative form, whose taller
        // units re-read fewer halo rows with as many waves (single images and batches
        // by keys of their own)
        const int cmin = batch ? tu.batch_coop_min_wy : tu.coop_min_wy;
        if (cmin > 0 && j.wy >= cmin && stream_two_level(j.wy) && j.hm != PASS_VHGW &&
            rows_aligned(j)) {
            TileJob c = j;
            c.coop = batch ? tu.batch_coop_waves : tu.coop_waves;
            c.TB = std::min(batch ? tu.batch_coop_rows : tu.coop_rows, (H + 7) / 8 * 8);
            if (!batch && tu.fit_units) c.TB = fit_rows(c.TB, H, c.tiles_x * c.coop);
            if (coop_lds_bytes(c) <= kCoopMaxLds) j = c;
        }
        j.tiles_y = (H + j.TB - 1) / j.TB;
        if ((int64_t)j.tiles_x * j.tiles_y > INT32_MAX - 4) return MORPH_EUNSUPPORTED;
        return MORPH_OK;
    }
    // tile shape
    int tw = plan && plan->tile_w > 0 ? plan->tile_w : 0;
    int tb = plan && plan->tile_h > 0 ? plan->tile_h : 0;
    if ((tw && tw % 4) || (tb && tb % 2)) return MORPH_EINVAL;
    if (!tw || !tb) {
        const int wm = std::max(j.wx, j.wy);
        for (const TileRule &r : tu.tiles)
            if (wm <= r.wmax) {
                // the tile input (tw + wx - 1 columns, plus up to 3 for the origin
                // rounded down to a quad) fills exactly tq quads
                // (but at least about twice the window wide, so that wide windows do
                // not leave a tile mostly halo)
                if (!tw)
                    tw = std::max(4 * r.tq - ((j.wx + 2 + 3) & ~3), (2 * j.wx + 3) & ~3);
                if (!tb) tb = r.tb;
                break;
            }
        if (!tw) tw = 120;
        if (!tb) tb = 64;
    }
    const int w4 = (W + 3) & ~3;
    tw = std::min(tw, std::max(4, w4));
    tb = std::min(tb, std::max(2, (H + 1) & ~1));
    for (;;) {
        j.TW = tw;
        j.TB = tb;
        // A: 16-bit rows covering the tile input columns (+ 3 for the origin rounded
        // down to a quad) and the columns a direct horizontal unit reads past the
        // last one; odd stride in dwords.  B: row pairs of the output columns (+ 3 for
        // the store's last quad); odd stride.
        const int acols = std::max(tw + j.wx - 1 + 3,
                                   j.hm == PASS_DIRECT
                                       ? tw + kDirectChunkX + std::max(j.wx, kDirectMax) + 3
                                       : 0) +
                          4;
        j.SA = ((acols + 1) / 2) | 1;
        j.SB = (j.hm == PASS_NONE) ? 0 : ((tw + 4) | 1);
        // vertical vHGW: split each block into runs so that a tile has about one run per
        // thread; run totals (2 dwords per run and quad) live where B is, before the
        // horizontal pass needs it
        j.vrun = 0;
        j.vtt = 0;
        if (j.vm == PASS_VHGW) {
            const int nq = (tw + j.wx - 1 + 3 + 3) / 4;           // quads, upper bound
            const int nbf = (tb + j.wy - 1 + j.wy - 1) / j.wy;    // blocks, upper bound
            int ns = std::max(1, (kThreads + nq * nbf - 1) / (nq * nbf));
            ns = std::min(ns, (j.wy + kVhgwBatch - 1) / kVhgwBatch);
            int run = (j.wy + ns - 1) / ns;
            run = (run + kVhgwBatch - 1) / kVhgwBatch * kVhgwBatch;
            ns = (j.wy + run - 1) / run;
            j.vrun = run;
            j.vtt = ns > 1 ? 2 * nq * nbf * ns : 0;
        }
        const int lds = lds_bytes(j);
        if (lds <= 64 * 1024) break;
        if (user_tile && lds <= kMaxLdsBytes) break;
        if (tb > 2) {
            tb = std::max(2, (tb / 2) & ~1);
        } else if (lds <= kMaxLdsBytes) {
            break;
        } else if (tw > 4) {
            tw = std::max(4, (tw / 2) & ~3);
        } else {
            return MORPH_EUNSUPPORTED; // the window's row segment does not fit in LDS
        }
    }
    j.tiles_x = (W + j.TW - 1) / j.TW;
    j.tiles_y = (H + j.TB - 1) / j.TB;
    // the kernels split work-unit indices u by a divisor d with a multiply-high,
    // exact while u * d < 2^32 (largest u is units - 1 of each loop)
    const uint64_t nq = (uint64_t)(j.TW + j.wx - 1 + 3 + 3) / 4, np = (uint64_t)(j.TB + 1) / 2;
    const uint64_t nrow_blocks = (uint64_t)j.TB + j.wy; // >= row chunks / blocks of any loop
    const uint64_t ncol_blocks = (uint64_t)j.TW + j.wx; // >= column chunks / blocks
    if (nq * nq * nrow_blocks >= (1ull << 32) || np * np * ncol_blocks >= (1ull << 32))
        return MORPH_EUNSUPPORTED;
    return MORPH_OK;
}

// The one-pass opening (opening) or closing of one image on the wave kernel's form,
// where it applies: rows aligned, effective windows up to kOcWaveMaxWx x kOcWaveMaxWy.
bool plan_openclose_wave(bool opening, int dtype, const void *src, void *dst, int H, int W,
                         size_t pitch, int wx, int wy, int ax, int ay, TileJob &j)
{
    if (ax < 0) ax = default_anchor(wx);
    if (ay < 0) ay = default_anchor(wy);
    const int axe = std::min(ax, W - 1), rxe = std::min(wx - 1 - ax, W - 1);
    const int aye = std::min(ay, H - 1), rye = std::min(wy - 1 - ay, H - 1);
    j = TileJob{};
    j.src = (const uint8_t *)src;
    j.dst = (uint8_t *)dst;
    j.H = H;
    j.W = W;
    j.pitch = j.dpitch = (int64_t)pitch;
    j.wx = axe + rxe + 1;
    j.wy = aye + rye + 1;
    j.ax = axe;
    j.ay = aye;
    j.op = opening ? 1 : 0;
    j.dtype = dtype;
    if (j.wx > kOcWaveMaxWx || j.wy > kOcWaveMaxWy || !rows_aligned(j)) return false;
    const DtypeTuning tu = tuning_for(dtype);
    j.hm = j.wx <= tu.oc_t_x ? PASS_DIRECT : PASS_DOUBLING;
    j.TW = 4 * strip_quads(W, oc_quads(j.wx));
    j.TB = std::min(j.wy > kDirectMax ? tu.oc_rows_tall : tu.oc_rows,
                    (H + kWaveRows - 1) / kWaveRows * kWaveRows);
    j.tiles_x = (W + j.TW - 1) / j.TW;
    if (tu.fit_units) j.TB = fit_rows(j.TB, H, j.tiles_x);
    j.tiles_y = (H + j.TB - 1) / j.TB;
    return (int64_t)j.tiles_x * j.tiles_y <= INT32_MAX - 4;
}

// keep: a later launch of the same call reads dst (an intermediate image)
int run_single(int op, int dtype, const void *src, void *dst, int H, int W, size_t pitch, int wx,
               int wy, int ax, int ay, const morph_plan *plan, hipStream_t stream,
               bool keep = false)
{
    TileJob j;
    int rc = plan_job(op, dtype, src, dst, H, W, pitch, pitch, wx, wy, ax, ay, plan, j);
    if (rc != MORPH_OK) return rc;
    j.keep = keep ? 1 : 0;
    hipError_t e = launch_tile_job(j, stream);
    if (e != hipSuccess) return hip_fail(e);
    return MORPH_OK;
}

} // namespace

namespace morph {
int record_hip_error(hipError_t e) { return hip_fail(e); }
} // namespace morph

// ---------------- C ABI ----------------
extern "C" {

// Morphological gradient: both extrema from one read where the wave kernel runs the
// job on aligned rows, else dilation into dst, erosion into the workspace and dst
// minus the workspace.
static int run_gradient(int dtype, const void *src, void *dst, int H, int W, size_t pitch,
                        int wx, int wy, int ax, int ay, const morph_plan *plan, void *workspace,
                        size_t ws_bytes, hipStream_t stream)
{
    TileJob j;
    int rc = plan_job(MORPH_OP_ERODE, dtype, src, dst, H, W, pitch, pitch, wx, wy, ax, ay, plan, j);
    if (rc != MORPH_OK) return rc;
    hipError_t e;
    if (j.kind == KIND_WAVE && !wave_tall(j) && j.hm != PASS_VHGW && job_rows_aligned(j)) {
        if ((e = launch_gradient_job(j, stream)) != hipSuccess) return hip_fail(e);
        return MORPH_OK;
    }
    const size_t span = image_span(H, W, pitch, dtype);
    if (!workspace || ws_bytes < morph_workspace_bytes(H, W, pitch, (int)elem_bytes(dtype)))
        return MORPH_ENOMEM;
    if (ranges_overlap(workspace, span, src, span) || ranges_overlap(workspace, span, dst, span))
        return MORPH_EALIAS;
    rc = run_single(MORPH_OP_DILATE, dtype, src, dst, H, W, pitch, wx, wy, ax, ay, plan, stream,
                    true);
    if (rc != MORPH_OK) return rc;
    rc = run_single(MORPH_OP_ERODE, dtype, src, workspace, H, W, pitch, wx, wy, ax, ay, plan,
                    stream, true);
    if (rc != MORPH_OK) return rc;
    if ((e = launch_subtract(workspace, dst, H, W, pitch, dtype, false, stream)) != hipSuccess)
        return hip_fail(e);
    return MORPH_OK;
}

int morph_apply(int op, int dtype, const void *src, void *dst, int H, int W, size_t pitch,
                int wx, int wy, int anchor_x, int anchor_y, int border, const morph_plan *plan,
                void *workspace, size_t ws_bytes, hipStream_t stream)
{
    if (op < MORPH_OP_ERODE || op > MORPH_OP_BLACKHAT) return MORPH_EINVAL;
    int rc = check_image(dtype, src, dst, H, W, pitch, wx, wy, anchor_x, anchor_y, border);
    if (rc != MORPH_OK || H == 0 || W == 0) return rc;
    const size_t span = image_span(H, W, pitch, dtype);
    if (ranges_overlap(src, span, dst, span)) return MORPH_EALIAS;
    if (op == MORPH_OP_ERODE || op == MORPH_OP_DILATE)
        return run_single(op, dtype, src, dst, H, W, pitch, wx, wy, anchor_x, anchor_y, plan,
                          stream);
    if (op == MORPH_OP_GRADIENT)
        return run_gradient(dtype, src, dst, H, W, pitch, wx, wy, anchor_x, anchor_y, plan,
                            workspace, ws_bytes, stream);
    // opening = dilate(erode(src)), closing = erode(dilate(src)) (§2): in one pass
    // where the wave kernel's form takes it (no plan asked for), else two launches
    // through the workspace
    const bool opens = op == MORPH_OP_OPEN || op == MORPH_OP_TOPHAT;
    // (top-hat: src - opening; black-hat: closing - src, one subtraction after)
    if (!plan && tuning_for(dtype).oc_one_pass) {
        TileJob oj;
        if (plan_openclose_wave(opens, dtype, src, dst, H, W, pitch, wx, wy, anchor_x, anchor_y,
                                oj)) {
            oj.keep = op == MORPH_OP_TOPHAT || op == MORPH_OP_BLACKHAT; // (subtraction reads dst)
            hipError_t e = launch_openclose_wave(oj, stream);
            if (e == hipSuccess && (op == MORPH_OP_TOPHAT || op == MORPH_OP_BLACKHAT))
                e = launch_subtract(src, dst, H, W, pitch, dtype, op == MORPH_OP_TOPHAT, stream);
            return e == hipSuccess ? MORPH_OK : hip_fail(e);
        }
    }
    if (!workspace || ws_bytes < morph_workspace_bytes(H, W, pitch, (int)elem_bytes(dtype)))
        return MORPH_ENOMEM;
    if (ranges_overlap(workspace, span, src, span) || ranges_overlap(workspace, span, dst, span))
        return MORPH_EALIAS;
    // (top-hat: src - opening; black-hat: closing - src)
    const int first = opens ? MORPH_OP_ERODE : MORPH_OP_DILATE;
    rc = run_single(first, dtype, src, workspace, H, W, pitch, wx, wy, anchor_x, anchor_y, plan,
                    stream, true);
    if (rc != MORPH_OK) return rc;
    rc = run_single(1 - first, dtype, workspace, dst, H, W, pitch, wx, wy, anchor_x, anchor_y,
                    plan, stream, op == MORPH_OP_TOPHAT || op == MORPH_OP_BLACKHAT);
    if (rc != MORPH_OK || op == MORPH_OP_OPEN || op == MORPH_OP_CLOSE) return rc;
    hipError_t e = launch_subtract(src, dst, H, W, pitch, dtype, op == MORPH_OP_TOPHAT, stream);
    return e == hipSuccess ? MORPH_OK : hip_fail(e);
}

#define MORPH_SINGLE(name, op, dt)                                                            \
    int name(const void *src, void *dst, int H, int W, size_t pitch, int wx, int wy, int ax,   \
             int ay, int border, hipStream_t stream)                                          \
    {                                                                                          \
        return morph_apply(op, dt, src, dst, H, W, pitch, wx, wy, ax, ay, border, nullptr,    \
                           nullptr, 0, stream);                                                \
    }
MORPH_SINGLE(morph_erode, MORPH_OP_ERODE, MORPH_U8)
MORPH_SINGLE(morph_dilate, MORPH_OP_DILATE, MORPH_U8)
MORPH_SINGLE(morph_erode_u16, MORPH_OP_ERODE, MORPH_U16)
MORPH_SINGLE(morph_dilate_u16, MORPH_OP_DILATE, MORPH_U16)
#undef MORPH_SINGLE

#define MORPH_COMPOSED(name, op, dt)                                                          \
    int name(const void *src, void *dst, int H, int W, size_t pitch, int wx, int wy, int ax,   \
             int ay, int border, void *ws, size_t ws_bytes, hipStream_t stream)               \
    {                                                                                          \
        return morph_apply(op, dt, src, dst, H, W, pitch, wx, wy, ax, ay, border, nullptr,    \
                           ws, ws_bytes, stream);                                              \
    }
MORPH_COMPOSED(morph_open, MORPH_OP_OPEN, MORPH_U8)
MORPH_COMPOSED(morph_close, MORPH_OP_CLOSE, MORPH_U8)
MORPH_COMPOSED(morph_open_u16, MORPH_OP_OPEN, MORPH_U16)
MORPH_COMPOSED(morph_close_u16, MORPH_OP_CLOSE, MORPH_U16)
MORPH_COMPOSED(morph_gradient, MORPH_OP_GRADIENT, MORPH_U8)
MORPH_COMPOSED(morph_gradient_u16, MORPH_OP_GRADIENT, MORPH_U16)
MORPH_COMPOSED(morph_tophat, MORPH_OP_TOPHAT, MORPH_U8)
MORPH_COMPOSED(morph_blackhat, MORPH_OP_BLACKHAT, MORPH_U8)
MORPH_COMPOSED(morph_tophat_u16, MORPH_OP_TOPHAT, MORPH_U16)
MORPH_COMPOSED(morph_blackhat_u16, MORPH_OP_BLACKHAT, MORPH_U16)
#undef MORPH_COMPOSED

static_assert(kOcMaxW == MORPH_OPENCLOSE_FUSED_MAX_W, "fused opening/closing window limit");
static_assert(kOcWaveMaxWx == MORPH_OPENCLOSE_ONE_PASS_MAX_WX &&
                  kOcWaveMaxWy == MORPH_OPENCLOSE_ONE_PASS_MAX_WY,
              "one-pass opening/closing window limits");

int morph_openclose_fused(int dtype, int opening, const void *src, void *dst, int H, int W,
                          size_t pitch, int wx, int wy, int anchor_x, int anchor_y, int border,
                          hipStream_t stream)
{
    int rc = check_image(dtype, src, dst, H, W, pitch, wx, wy, anchor_x, anchor_y, border);
    if (rc != MORPH_OK || H == 0 || W == 0) return rc;
    const size_t span = image_span(H, W, pitch, dtype);
    if (ranges_overlap(src, span, dst, span)) return MORPH_EALIAS;
    // the wave kernel's form where it applies, else the workgroup-tile kernel
    TileJob oj;
    if (plan_openclose_wave(opening != 0, dtype, src, dst, H, W, pitch, wx, wy, anchor_x, anchor_y,
                            oj)) {
        hipError_t e = launch_openclose_wave(oj, stream);
        return e == hipSuccess ? MORPH_OK : hip_fail(e);
    }
    if (wx > kOcMaxW || wy > kOcMaxW) return MORPH_EUNSUPPORTED;
    const int ax = anchor_x < 0 ? default_anchor(wx) : anchor_x;
    const int ay = anchor_y < 0 ? default_anchor(wy) : anchor_y;
    hipError_t e = launch_openclose(src, dst, H, W, pitch, wx, wy, ax, ay, opening != 0, dtype,
                                    stream);
    return e == hipSuccess ? MORPH_OK : hip_fail(e);
}

size_t morph_workspace_bytes(int H, int W, size_t pitch, int elem_bytes_)
{
    (void)elem_bytes_;
    if (H <= 0 || W <= 0) return 0;
    return (size_t)H * pitch;
}

int morph_load_tuning(const char *json_path)
{
    if (!json_path) {
        std::lock_guard<std::mutex> lk(g_tuning_mu);
        g_tuning[0] = k_builtin_tuning[0];
        g_tuning[1] = k_builtin_tuning[1];
        return MORPH_OK;
    }
    FILE *f = std::fopen(json_path, "rb");
    if (!f) return MORPH_EINVAL;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    std::fclose(f);
    JVal root;
    JParser jp{text.data(), text.data() + text.size()};
    if (!jp.parse(root) || root.k != JVal::OBJ) return MORPH_EINVAL;
    DtypeTuning next[2];
    {
        std::lock_guard<std::mutex> lk(g_tuning_mu);
        next[0] = g_tuning[0];
        next[1] = g_tuning[1];
    }
    const char *keys[2] = {"u8", "u16"};
    for (int d = 0; d < 2; d++) {
        auto it = root.obj.find(keys[d]);
        if (it != root.obj.end() && !read_dtype_tuning(it->second, next[d])) return MORPH_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    g_tuning[0] = next[0];
    g_tuning[1] = next[1];
    return MORPH_OK;
}

int morph_get_thresholds(int dtype, int *t_x, int *t_y)
{
    if (dtype != MORPH_U8 && dtype != MORPH_U16) return MORPH_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    if (t_x) *t_x = g_tuning[dtype].t_x;
    if (t_y) *t_y = g_tuning[dtype].t_y;
    return MORPH_OK;
}

int morph_set_thresholds(int dtype, int t_x, int t_y)
{
    if (dtype != MORPH_U8 && dtype != MORPH_U16) return MORPH_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    if (t_x > 0) g_tuning[dtype].t_x = t_x;
    if (t_y > 0) g_tuning[dtype].t_y = t_y;
    return MORPH_OK;
}

int morph_resolve_plan(int dtype, int H, int W, int wx, int wy, morph_plan *plan)
{
    if (!plan || H <= 0 || W <= 0 || wx < 1 || wy < 1) return MORPH_EINVAL;
    if (dtype != MORPH_U8 && dtype != MORPH_U16) return MORPH_EUNSUPPORTED;
    TileJob j;
    const morph_plan in = *plan;
    const size_t p = (size_t)W * elem_bytes(dtype);
    int rc = plan_job(MORPH_OP_ERODE, dtype, (const void *)16, (void *)16, H, W, p, p, wx, wy, -1,
                      -1, &in, j, in.batch != 0);
    if (rc != MORPH_OK) return rc;
    plan->method_x = j.hm == PASS_NONE        ? MORPH_METHOD_AUTO
                     : j.hm == PASS_DIRECT   ? MORPH_METHOD_DIRECT
                     : j.hm == PASS_DOUBLING ? MORPH_METHOD_DOUBLING
                                             : MORPH_METHOD_VHGW;
    plan->method_y = (j.wy == 1) ? MORPH_METHOD_AUTO
                                 : (j.vm == PASS_DIRECT ? MORPH_METHOD_DIRECT : MORPH_METHOD_VHGW);
    plan->tile_w = j.TW;
    plan->tile_h = j.TB;
    // (KernelKind values are the MORPH_KERNEL_* codes)
    plan->kernel = j.coop ? MORPH_KERNEL_STREAM_COOP : j.kind;
    return MORPH_OK;
}

const char *morph_strerror(int status)
{
    switch (status) {
    case MORPH_OK: return "ok";
    case MORPH_EINVAL: return "invalid argument";
    case MORPH_EALIAS: return "source and destination overlap";
    case MORPH_EUNSUPPORTED: return "unsupported border, dtype or window";
    case MORPH_EHIP: return "HIP call failed";
    case MORPH_ENOMEM: return "workspace or table too small";
    default: return "unknown status";
    }
}

// ---------------- transposes (§4; their use in §1) ----------------
static int transpose_image(int dtype, const void *src, void *dst, int H, int W,
                           size_t src_pitch, size_t dst_pitch, hipStream_t stream)
{
    const size_t es = elem_bytes(dtype);
    if (H < 0 || W < 0) return MORPH_EINVAL;
    if (H == 0 || W == 0) return MORPH_OK;
    if (!src || !dst) return MORPH_EINVAL;
    if (src_pitch < (size_t)W * es || src_pitch % es || dst_pitch < (size_t)H * es ||
        dst_pitch % es)
        return MORPH_EINVAL;
    if (src_pitch > (size_t)1 << 40 || dst_pitch > (size_t)1 << 40) return MORPH_EINVAL;
    if (es == 2 && (((uintptr_t)src | (uintptr_t)dst) & 1)) return MORPH_EINVAL;
    const size_t sspan = (size_t)(H - 1) * src_pitch + (size_t)W * es;
    const size_t dspan = (size_t)(W - 1) * dst_pitch + (size_t)H * es;
    if (ranges_overlap(src, sspan, dst, dspan)) return MORPH_EALIAS;
    const hipError_t e = launch_transpose(src, dst, H, W, src_pitch, dst_pitch, dtype, stream);
    return e == hipSuccess ? MORPH_OK : hip_fail(e);
}

int morph_transpose(const void *src, void *dst, int H, int W, size_t src_pitch,
                    size_t dst_pitch, hipStream_t stream)
{
    return transpose_image(MORPH_U8, src, dst, H, W, src_pitch, dst_pitch, stream);
}

int morph_transpose_u16(const void *src, void *dst, int H, int W, size_t src_pitch,
                        size_t dst_pitch, hipStream_t stream)
{
    return transpose_image(MORPH_U16, src, dst, H, W, src_pitch, dst_pitch, stream);
}

int morph_transpose_blocks(const void *src, void *dst, int64_t n_blocks, int dtype,
                           hipStream_t stream)
{
    if (dtype != MORPH_U8 && dtype != MORPH_U16) return MORPH_EUNSUPPORTED;
    if (n_blocks < 0 || n_blocks > ((int64_t)1 << 34)) return MORPH_EINVAL;
    if (n_blocks == 0) return MORPH_OK;
    if (!src || !dst || (((uintptr_t)src | (uintptr_t)dst) & 3)) return MORPH_EINVAL;
    const size_t span = (size_t)n_blocks * (dtype == MORPH_U8 ? 256 : 128);
    if (ranges_overlap(src, span, dst, span)) return MORPH_EALIAS;
    const hipError_t e = launch_transpose_blocks(src, dst, n_blocks, dtype, stream);
    return e == hipSuccess ? MORPH_OK : hip_fail(e);
}

int morph_last_hip_error(void) { return g_last_hip_error; }

const char *morph_version(void) { return "morph-gfx950 0.1"; }

// ---------------- batched persistent launch ----------------
// Jobs are grouped by element type and row alignment (one persistent kernel per
// group); within a group, tiles are numbered by a prefix sum over the jobs.
struct BatchGroup {
    int job0 = 0, njobs = 0; // jobs [job0, job0 + njobs) of the (group-sorted) table
    int64_t tiles = 0;
    int lds = 0, grid = 0, dtype = 0, kind = 0, variant = 0, phase = 0;
    int waves = 0; // the cooperative form's waves a unit (streaming variant 2)
    bool aligned = true;
};

// A job of the table that reads or writes an intermediate image in the enqueue
// workspace: its pointer is set to workspace + offset when the workspace is bound.
struct WsPatch {
    int job;        // index into the job table
    bool writes;    // first operation (dst = intermediate) or second (src = intermediate)
    size_t offset;  // bytes from the workspace start
};

// groups: kernel kind x element type x row alignment, for the streaming kernel its
// two vertical forms (LDS ring for wy <= kStreamRingMaxWy, run totals above) and for
// the wave kernel its two forms (vertical windows up to kDirectMax, tall beyond)
// group classes: tile, wave, streaming (ring), streaming (run totals), wide rows, wave
// (tall), streaming (cooperative form)
static constexpr int kGroupClasses = kKinds + 3;
static constexpr int kClassRows = kKinds;          // wide rows
static constexpr int kClassWaveTall = kKinds + 1;  // tall wave units
static constexpr int kClassCoop = kKinds + 2;      // cooperative streaming units
static constexpr int kPhaseGroups = 4 * kGroupClasses;
// an opening or closing descriptor is two jobs: its first operation (src into the
// workspace) in phase 0 with every erosion and dilation, its second (workspace into
// dst) in phase 1, launched after all of phase 0
static constexpr int kPhases = 2;
static constexpr int kBatchGroups = kPhases * kPhaseGroups;

struct morph_batch {
    int max_images = 0;
    int64_t max_tiles = 0;
    // the three tables of a batch, packed into one device block (and one pinned
    // staging block, so that set() copies them with one transfer): laid out anew by
    // each set() for its number of jobs, each table on a 256-byte boundary
    uint8_t *d_tables = nullptr, *h_tables = nullptr;
    TileJob *d_jobs = nullptr;            // the job table
    int64_t *d_tile_start = nullptr;      // per group: njobs + 1 prefix sums
    int32_t *d_tile_job = nullptr;        // per group: job (within the group) of each tile
    TileJob *h_jobs = nullptr;            // their places in the staging block
    int64_t *h_tile_start = nullptr;
    int32_t *h_tile_job = nullptr;
    unsigned long long *d_counter = nullptr; // per group: next tile, finished workgroups
    std::vector<BatchGroup> groups;
    int64_t n_tiles = -1;
    // captured graph of the group launches, valid for one stream and one layout
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t graph_stream = nullptr;
    bool graph_valid = false;
    // the pinned staging tables are copied asynchronously: set() waits for the
    // previous copy before it overwrites them
    hipEvent_t staged = nullptr;
    bool staged_pending = false;
    // openings and closings: intermediates in the caller's workspace
    std::vector<WsPatch> ws_patch;
    size_t ws_needed = 0;          // bytes of workspace the current batch needs
    const void *ws_bound = nullptr; // workspace the device job table points into
    int n_jobs = 0;                 // jobs in the table
    TileJob *h_jobs_ws = nullptr;  // pinned staging of the job table with the pointers set
    hipEvent_t ws_staged = nullptr; // its copy to the device
    bool ws_staged_pending = false;
};


static int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 256;
    return cus > 0 ? cus : 256;
}

// Lay the batch's tables out for `njobs` jobs in `ngroups` groups and `tiles` tiles:
// the job table, then the tile starts (njobs + ngroups), then the tile jobs, each on
// a 256-byte boundary; point the device and staging pointers there (once the blocks
// exist) and return the bytes the three take.
static size_t table_layout(morph_batch *b, size_t njobs, size_t ngroups, int64_t tiles)
{
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_start = up(sizeof(TileJob) * njobs);
    const size_t o_tjob = up(o_start + sizeof(int64_t) * (njobs + ngroups));
    if (b->d_tables && b->h_tables) {
        b->d_jobs = (TileJob *)b->d_tables;
        b->d_tile_start = (int64_t *)(b->d_tables + o_start);
        b->d_tile_job = (int32_t *)(b->d_tables + o_tjob);
        b->h_jobs = (TileJob *)b->h_tables;
        b->h_tile_start = (int64_t *)(b->h_tables + o_start);
        b->h_tile_job = (int32_t *)(b->h_tables + o_tjob);
    }
    return o_tjob + sizeof(int32_t) * (size_t)tiles;
}

static void drop_graph(morph_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_valid = false;
}

int morph_batch_create(int max_images, int64_t max_tiles, morph_batch_t *out)
{
    if (!out || max_images < 1 || max_tiles < 1 || max_tiles > INT32_MAX - 4) return MORPH_EINVAL;
    *out = nullptr;
    morph_batch *b = new morph_batch();
    b->max_images = max_images;
    b->max_tiles = max_tiles;
    const size_t njobs = (size_t)kPhases * max_images; // an opening/closing is two jobs
    const size_t ncount = 2 * kBatchGroups;
    const size_t bytes = table_layout(b, njobs, kBatchGroups, max_tiles);
    hipError_t e;
    if ((e = hipMalloc((void **)&b->d_tables, bytes)) != hipSuccess ||
        (e = hipHostMalloc((void **)&b->h_tables, bytes)) != hipSuccess ||
        (e = hipMalloc((void **)&b->d_counter, sizeof(unsigned long long) * ncount)) !=
            hipSuccess ||
        (e = hipMemset(b->d_counter, 0, sizeof(unsigned long long) * ncount)) != hipSuccess ||
        (e = hipHostMalloc((void **)&b->h_jobs_ws, sizeof(TileJob) * njobs)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&b->ws_staged, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming)) != hipSuccess) {
        morph_batch_destroy(b);
        return hip_fail(e);
    }
    (void)table_layout(b, njobs, kBatchGroups, max_tiles); // (places the pointers)
    *out = b;
    return MORPH_OK;
}

// Group index of a job: (dtype, alignment) in the low two bits; above them the
// kernel kind, the streaming kernel split by ring size.
static int group_of(const TileJob &j, int phase)
{
    int k = j.kind;
    if (j.kind == KIND_STREAM && j.coop) k = kClassCoop;
    else if (j.kind == KIND_STREAM && stream_two_level(j.wy)) k = KIND_STREAM + 1;
    else if (j.kind == KIND_ROWS) k = kClassRows;
    else if (wave_tall(j)) k = kClassWaveTall;
    return phase * kPhaseGroups + 4 * k + 2 * j.dtype + (job_rows_aligned(j) ? 0 : 1);
}

// Launch order of the groups: phase 0 before phase 1; within a phase the streaming
// groups (run totals, then ring), then the tile, wave and wide-row groups.
static int group_order(int gi)
{
    static const int order[kGroupClasses] = {kClassCoop, KIND_STREAM + 1, KIND_STREAM,
                                             kClassWaveTall, KIND_TILE, KIND_WAVE, kClassRows};
    const int ph = gi / kPhaseGroups, r = gi % kPhaseGroups;
    return ph * kPhaseGroups + 4 * order[r / 4] + r % 4;
}

// Row pitch of an intermediate image in the workspace: whole 64-byte granules.
static size_t ws_pitch(int W, int dtype) { return ((size_t)W * elem_bytes(dtype) + 63) & ~(size_t)63; }

int morph_batch_set(morph_batch_t b, const morph_desc *descs, int n, hipStream_t stream)
{
    if (!b || n < 0 || (n > 0 && !descs)) return MORPH_EINVAL;
    if (n > b->max_images) return MORPH_ENOMEM;
    if (b->staged_pending) {
        hipError_t e = hipEventSynchronize(b->staged);
        if (e != hipSuccess) return hip_fail(e);
        b->staged_pending = false;
    }
    std::vector<TileJob> jobs[kBatchGroups];
    // per group, for each job: the workspace offset of its intermediate and whether
    // it writes (first operation) or reads it (second); -1 = none
    std::vector<std::pair<int64_t, bool>> wsrole[kBatchGroups];
    size_t ws_total = 0;
    for (int i = 0; i < n; i++) {
        const morph_desc &d = descs[i];
        if (d.op < MORPH_OP_ERODE || d.op > MORPH_OP_CLOSE) return MORPH_EINVAL;
        if (d.pitch < 0 || d.dst_pitch < 0) return MORPH_EINVAL;
        const size_t dp = d.dst_pitch ? (size_t)d.dst_pitch : (size_t)d.pitch;
        int rc = check_image(d.dtype, d.src, d.dst, d.H, d.W, (size_t)d.pitch, d.wx, d.wy, d.ax,
                             d.ay, MORPH_BORDER_NEUTRAL);
        if (rc != MORPH_OK) return rc;
        if (d.H == 0 || d.W == 0) continue;
        if (dp < (size_t)d.W * elem_bytes(d.dtype) || dp % elem_bytes(d.dtype)) return MORPH_EINVAL;
        if (ranges_overlap(d.src, image_span(d.H, d.W, (size_t)d.pitch, d.dtype), d.dst,
                           image_span(d.H, d.W, dp, d.dtype)))
            return MORPH_EALIAS;
        TileJob j;
        if (d.op == MORPH_OP_ERODE || d.op == MORPH_OP_DILATE) {
            rc = plan_job(d.op, d.dtype, d.src, d.dst, d.H, d.W, (size_t)d.pitch, dp, d.wx, d.wy,
                          d.ax, d.ay, nullptr, j, true);
            if (rc != MORPH_OK) return rc;
            const int g = group_of(j, 0);
            jobs[g].push_back(j);
            wsrole[g].push_back({-1, false});
            continue;
        }
        // opening = dilate(erode(src)), closing = erode(dilate(src)) (§2): the first
        // operation into an intermediate in the workspace (placed when the workspace
        // is bound at enqueue; null until then), the second from it into dst
        const int first = d.op == MORPH_OP_OPEN ? MORPH_OP_ERODE : MORPH_OP_DILATE;
        const size_t wp = ws_pitch(d.W, d.dtype);
        const size_t off = ws_total;
        ws_total += ((size_t)d.H * wp + 255) & ~(size_t)255;
        rc = plan_job(first, d.dtype, d.src, nullptr, d.H, d.W, (size_t)d.pitch, wp, d.wx, d.wy,
                      d.ax, d.ay, nullptr, j, true);
        if (rc != MORPH_OK) return rc;
        int g = group_of(j, 0);
        jobs[g].push_back(j);
        wsrole[g].push_back({(int64_t)off, true});
        rc = plan_job(1 - first, d.dtype, nullptr, d.dst, d.H, d.W, wp, dp, d.wx, d.wy, d.ax,
                      d.ay, nullptr, j, true);
        if (rc != MORPH_OK) return rc;
        g = group_of(j, 1);
        jobs[g].push_back(j);
        wsrole[g].push_back({(int64_t)off, false});
    }
    // a batch of few or small images (a serving loop's micro-batch, often one image)
    // would have too few wave and streaming units to fill the GPU: as for a single
    // image, shorten them until the batch has about kUnitTarget
    {
        int64_t units = 0, rows_strips = 0;
        for (int g = 0; g < kBatchGroups; g++)
            for (const TileJob &j : jobs[g])
                if ((j.kind == KIND_WAVE || j.kind == KIND_STREAM) && tuning_for(j.dtype).fit_units) {
                    units += (int64_t)j.tiles_x * j.tiles_y;
                    rows_strips += (int64_t)j.H * j.tiles_x;
                }
        if (units > 0 && units < kUnitTarget) {
            const int64_t need = (rows_strips + kUnitTarget - 1) / kUnitTarget;
            const int tb = (int)std::min<int64_t>((need + 7) / 8 * 8, INT32_MAX);
            auto fitted = [&](const TileJob &j) { return std::max(std::min(j.TB, 8), std::min(j.TB, tb)); };
            // (only if the batch's tile table still holds the longer list)
            int64_t total = 0;
            for (int g = 0; g < kBatchGroups; g++)
                for (const TileJob &j : jobs[g]) {
                    const bool fit = (j.kind == KIND_WAVE || j.kind == KIND_STREAM) &&
                                     tuning_for(j.dtype).fit_units;
                    total += (int64_t)j.tiles_x * (fit ? (j.H + fitted(j) - 1) / fitted(j) : j.tiles_y);
                }
            if (total <= b->max_tiles)
                for (int g = 0; g < kBatchGroups; g++)
                    for (TileJob &j : jobs[g])
                        if ((j.kind == KIND_WAVE || j.kind == KIND_STREAM) &&
                            tuning_for(j.dtype).fit_units) {
                            j.TB = fitted(j);
                            j.tiles_y = (j.H + j.TB - 1) / j.TB;
                        }
        }
    }
    // from here on the staged tables change: until this set succeeds the batch has no
    // work (enqueue and launch return MORPH_EINVAL)
    b->n_tiles = -1;
    b->ws_needed = 0;
    b->ws_bound = nullptr;
    // the tables laid out for this batch's jobs, groups and tiles (within the
    // capacity: at most kPhases x max_images jobs, kBatchGroups groups, max_tiles)
    size_t n_all = 0, n_groups = 0;
    int64_t t_all = 0;
    for (int g = 0; g < kBatchGroups; g++) {
        n_all += jobs[g].size();
        n_groups += jobs[g].empty() ? 0 : 1;
        for (const TileJob &j : jobs[g]) t_all += (int64_t)j.tiles_x * j.tiles_y;
    }
    if (t_all > b->max_tiles) return MORPH_ENOMEM;
    const size_t table_bytes = table_layout(b, n_all, n_groups, t_all);
    std::vector<BatchGroup> groups;
    std::vector<WsPatch> patches;
    int64_t tiles = 0;
    int m = 0, starts = 0;
    const int cus = device_cus();
    for (int gi = 0; gi < kBatchGroups; gi++) {
        // the streaming groups first, then the rest
        const int g = group_order(gi);
        if (jobs[g].empty()) continue;
        BatchGroup G;
        G.job0 = m;
        G.njobs = (int)jobs[g].size();
        G.kind = jobs[g][0].kind;
        G.dtype = jobs[g][0].dtype;
        G.aligned = job_rows_aligned(jobs[g][0]);
        // streaming: 1 run totals, 2 the cooperative form; wave: 1 the tall form
        G.variant = (G.kind == KIND_STREAM && jobs[g][0].coop) ? 2
                    : ((G.kind == KIND_STREAM && stream_two_level(jobs[g][0].wy)) ||
                       wave_tall(jobs[g][0]))
                        ? 1
                        : 0;
        G.waves = jobs[g][0].coop;
        G.phase = g / kPhaseGroups;
        int64_t t = 0;
        for (size_t q = 0; q < jobs[g].size(); q++) {
            const TileJob &j = jobs[g][q];
            if (wsrole[g][q].first >= 0)
                patches.push_back(WsPatch{m, wsrole[g][q].second, (size_t)wsrole[g][q].first});
            b->h_tile_start[starts++] = t;
            b->h_jobs[m++] = j;
            t += (int64_t)j.tiles_x * j.tiles_y;
            G.lds = std::max(G.lds, lds_bytes(j));
        }
        b->h_tile_start[starts++] = t;
        G.tiles = t;
        if (G.kind == KIND_WAVE || G.kind == KIND_ROWS) {
            // one wave per unit, four per workgroup: the grid covers every unit
            G.grid = (int)std::max<int64_t>((t + 3) / 4, 1);
        } else if (G.kind == KIND_STREAM) {
            // one workgroup per unit (single-wave, or the cooperative form's)
            G.grid = (int)std::max<int64_t>(t, 1);
        } else {
            const int per_cu = std::max(1, std::min(8, kMaxLdsBytes / std::max(G.lds + 64, 1)));
            G.grid = (int)std::min<int64_t>((int64_t)cus * per_cu, std::max<int64_t>(t, 1));
        }
        tiles += t;
        groups.push_back(G);
    }
    if (tiles > b->max_tiles) return MORPH_ENOMEM;
    {
        int64_t at = 0;
        for (const BatchGroup &G : groups)
            for (int jj = 0; jj < G.njobs; jj++) {
                const TileJob &j = b->h_jobs[G.job0 + jj];
                const int64_t nt = (int64_t)j.tiles_x * j.tiles_y;
                for (int64_t k = 0; k < nt; k++) b->h_tile_job[at++] = jj;
            }
    }
    const bool same_layout = b->graph_valid && groups.size() == b->groups.size() &&
        std::equal(groups.begin(), groups.end(), b->groups.begin(),
                   [](const BatchGroup &x, const BatchGroup &y) {
                       return x.job0 == y.job0 && x.njobs == y.njobs && x.tiles == y.tiles &&
                              x.lds == y.lds && x.grid == y.grid && x.dtype == y.dtype &&
                              x.aligned == y.aligned && x.kind == y.kind &&
                              x.variant == y.variant && x.phase == y.phase && x.waves == y.waves;
                   });
    if (!same_layout) drop_graph(b);
    b->groups = groups;
    b->n_jobs = m;
    b->ws_patch = patches;
    hipError_t e;
    if (m > 0) {
        // the three tables in one transfer
        if ((e = hipMemcpyAsync(b->d_tables, b->h_tables, table_bytes, hipMemcpyHostToDevice,
                                stream)) != hipSuccess)
            return hip_fail(e);
        if ((e = hipEventRecord(b->staged, stream)) != hipSuccess) return hip_fail(e);
        b->staged_pending = true;
    }
    b->n_tiles = tiles;
    b->ws_needed = ws_total; // (the table just copied points into no workspace yet)
    return MORPH_OK;
}

// Class of a group in a fused dispatch (-1: launched on its own).
static int fused_class(const BatchGroup &G)
{
    if (!tuning_for(G.dtype).fuse) return -1;
    if (G.kind == KIND_STREAM && G.variant == 2) return -1; // (workgroups of several waves)
    if (G.kind == KIND_STREAM) return G.variant ? 0 : 1;
    return (G.kind == KIND_WAVE && !G.variant) ? 2 : -1;
}

// The wave and streaming groups of each element type and row alignment as one
// fused dispatch (see launch_fused), then the other groups' kernels, one after the
// other on the caller's stream (running the groups side by side on forked streams
// measured no faster on the benchmark batch; fusing them does).
static hipError_t launch_groups(morph_batch *b, hipStream_t stream)
{
    int start = 0;
    int64_t tstart = 0;
    std::vector<BatchTables> tabs(b->groups.size());
    for (size_t g = 0; g < b->groups.size(); g++) {
        const BatchGroup &G = b->groups[g];
        tabs[g] = BatchTables{b->d_jobs + G.job0, b->d_tile_start + start, b->d_tile_job + tstart,
                              G.njobs, G.tiles, b->d_counter + 2 * g};
        start += G.njobs + 1;
        tstart += G.tiles;
    }
    for (int ph = 0; ph < kPhases; ph++) {
    for (int dt = 0; dt < 2; dt++)
        for (int al = 0; al < 2; al++) {
            FusedTables ft{};
            int64_t n[kFusedClasses] = {0, 0, 0};
            int lds = 0;
            for (size_t g = 0; g < b->groups.size(); g++) {
                const BatchGroup &G = b->groups[g];
                const int c = fused_class(G);
                if (c < 0 || G.phase != ph || G.dtype != dt || G.aligned != (al == 0)) continue;
                ft.g[c] = tabs[g];
                n[c] = G.tiles;
                lds = std::max(lds, G.lds);
            }
            if (n[0] + n[1] + n[2] == 0) continue;
            ft.b0[0] = 0;
            for (int c = 0; c < kFusedClasses; c++) {
                const int64_t nb = ft.b0[c] + (n[c] + 7) / 8 * 8;
                if (nb > INT32_MAX) return hipErrorInvalidValue;
                ft.b0[c + 1] = (int32_t)nb;
            }
            hipError_t e = launch_fused(ft, dt, al == 0, lds, stream);
            if (e != hipSuccess) return e;
        }
    for (size_t g = 0; g < b->groups.size(); g++) {
        const BatchGroup &G = b->groups[g];
        if (fused_class(G) >= 0 || G.phase != ph) continue;
        hipError_t e = launch_batch(tabs[g], G.kind, G.variant, G.waves, G.dtype, G.aligned, G.grid,
                                    G.lds, stream);
        if (e != hipSuccess) return e;
    }
    }
    return hipSuccess;
}

// Kernel dispatches launch_groups makes: per phase, one per element type and row
// alignment with fused units, and one per other group.
static int count_dispatches(const morph_batch *b)
{
    int n = 0;
    bool fused[kPhases][2][2] = {};
    for (const BatchGroup &G : b->groups) {
        if (fused_class(G) < 0) n++;
        else if (!fused[G.phase][G.dtype][G.aligned ? 0 : 1]) {
            fused[G.phase][G.dtype][G.aligned ? 0 : 1] = true;
            n++;
        }
    }
    return n;
}

// Point the intermediates of the batch's openings and closings into `workspace`:
// check it (size, no overlap with any image of the batch), write the pointers into
// the staged job table and copy it to the device on `stream`, ahead of the launch.
static int bind_workspace(morph_batch *b, void *workspace, size_t ws_bytes, hipStream_t stream)
{
    if (b->ws_needed == 0) return MORPH_OK;
    if (!workspace || ws_bytes < b->ws_needed) return MORPH_ENOMEM;
    if (workspace == b->ws_bound) return MORPH_OK;
    // (h_jobs holds the images' own pointers, null where an intermediate goes)
    for (int i = 0; i < b->n_jobs; i++) {
        const TileJob &j = b->h_jobs[i];
        const size_t es = elem_bytes(j.dtype);
        if ((j.src && ranges_overlap(workspace, b->ws_needed, j.src,
                                     (size_t)(j.H - 1) * j.pitch + (size_t)j.W * es)) ||
            (j.dst && ranges_overlap(workspace, b->ws_needed, j.dst,
                                     (size_t)(j.H - 1) * j.dpitch + (size_t)j.W * es)))
            return MORPH_EALIAS;
    }
    hipError_t e;
    // a staging buffer of its own, so that binding never waits for set()'s copy
    if (b->ws_staged_pending) {
        if ((e = hipEventSynchronize(b->ws_staged)) != hipSuccess) return hip_fail(e);
        b->ws_staged_pending = false;
    }
    std::memcpy(b->h_jobs_ws, b->h_jobs, sizeof(TileJob) * b->n_jobs);
    for (const WsPatch &p : b->ws_patch) {
        uint8_t *ptr = (uint8_t *)workspace + p.offset;
        if (p.writes) b->h_jobs_ws[p.job].dst = ptr;
        else b->h_jobs_ws[p.job].src = ptr;
    }
    if ((e = hipMemcpyAsync(b->d_jobs, b->h_jobs_ws, sizeof(TileJob) * b->n_jobs,
                            hipMemcpyHostToDevice, stream)) != hipSuccess)
        return hip_fail(e);
    if ((e = hipEventRecord(b->ws_staged, stream)) != hipSuccess) return hip_fail(e);
    b->ws_staged_pending = true;
    b->ws_bound = workspace;
    return MORPH_OK;
}

int morph_batch_enqueue(morph_batch_t b, void *workspace, size_t ws_bytes, hipStream_t stream)
{
    if (!b || b->n_tiles < 0) return MORPH_EINVAL;
    if (b->n_tiles == 0) return MORPH_OK;
    int rc = bind_workspace(b, workspace, ws_bytes, stream);
    if (rc != MORPH_OK) return rc;
    hipError_t e;
    // The legacy null stream cannot be captured, and a batch of one dispatch gains
    // nothing from a graph (a one-node graph's replay measured ~4% slower than the
    // dispatch itself on the 512-image batch): launch directly.
    if (stream == nullptr || count_dispatches(b) <= 1) {
        if ((e = launch_groups(b, stream)) != hipSuccess) return hip_fail(e);
        return MORPH_OK;
    }
    if (!(b->graph_valid && b->graph_stream == stream)) {
        drop_graph(b);
        if ((e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(e);
        hipError_t le = launch_groups(b, stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(stream, &g);
        if (le != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(le);
        }
        if (e != hipSuccess) return hip_fail(e);
        b->graph = g;
        if ((e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
            b->exec = nullptr;
            drop_graph(b);
            return hip_fail(e);
        }
        b->graph_stream = stream;
        b->graph_valid = true;
    }
    if ((e = hipGraphLaunch(b->exec, stream)) != hipSuccess) return hip_fail(e);
    return MORPH_OK;
}

int morph_batch_launch(morph_batch_t b, void *workspace, size_t ws_bytes, hipStream_t stream)
{
    if (!b || b->n_tiles < 0) return MORPH_EINVAL;
    if (b->n_tiles == 0) return MORPH_OK;
    int rc = bind_workspace(b, workspace, ws_bytes, stream);
    if (rc != MORPH_OK) return rc;
    hipError_t e = launch_groups(b, stream);
    return e == hipSuccess ? MORPH_OK : hip_fail(e);
}

int64_t morph_batch_tiles(morph_batch_t b) { return b ? b->n_tiles : -1; }

size_t morph_batch_workspace_bytes(morph_batch_t b) { return b ? b->ws_needed : 0; }

int morph_batch_destroy(morph_batch_t b)
{
    if (!b) return MORPH_EINVAL;
    drop_graph(b);
    if (b->staged) (void)hipEventDestroy(b->staged);
    if (b->ws_staged) (void)hipEventDestroy(b->ws_staged);
    if (b->h_jobs_ws) (void)hipHostFree(b->h_jobs_ws);
    if (b->d_tables) (void)hipFree(b->d_tables);
    if (b->h_tables) (void)hipHostFree(b->h_tables);
    if (b->d_counter) (void)hipFree(b->d_counter);
    delete b;
    return MORPH_OK;
}

} // extern "C"
